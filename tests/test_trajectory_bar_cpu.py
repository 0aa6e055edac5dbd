"""The segment bars of the FP32 trajectory tests are discriminating (CPU only).

The GPU tests compare SEGMENT-step stretches of a run, re-anchored at a state
the GPU reached, with the oracle started from that state, ion by ion against
FACTOR times the envelope of the oracle's own run under velocity kicks of
dt M1 A_i per step (tests/trajectory_bar.py).  Here the oracle stands in for
the GPU: mistakes of the kind a wrong kernel would make are planted in an
oracle run (a wrong bath seed, swapped species, a beam rate off by 0.1 %, the
isotropic damping off by 0.1 %, one ion's body id changed), and each must move
the segment by at least 10 bars at the reference force error M1_REF.  A second
realisation of the kicks themselves (an FP32-size force error of other
directions) stays within the bars.
"""
from __future__ import annotations

import numpy as np
import pytest

import lion_inputs as li
from tests import trajectory_bar as tb

SEG = tb.SEGMENT


def _trap(oracle, spec):
    V0, U0 = oracle.voltages_for(spec.q_x, spec.a_x, spec.ref_mass, spec.ref_charge, spec.omega,
                                 spec.r0, spec.z0, spec.kappa)
    return oracle.Trap(V0=V0, Omega=spec.omega, U0=U0, R0=spec.r0, Z0=spec.z0, kappa=spec.kappa)


@pytest.fixture(scope="module")
def cooled(oracle_mod):
    """The cooled 700-ion cloud of the GPU cooling test, run by the oracle to
    step 120 (where the GPU test re-anchors a segment), its SEG-step segment
    and the kicked envelope at M1_REF."""
    from tests.test_gpu_cooling import BATHS, BEAMS

    w = li.random_cloud(700, seed=41, sigma=200e-6, light_fraction=0.3)
    sp = (w.mass < 30 * li.AMU).astype(np.int32)
    spec = w.traps[0]
    tr = _trap(oracle_mod, spec)
    dt, k0 = spec.dt, 120
    s = oracle_mod.step_cooled(w.state(), w.charge, w.mass, sp, tr, spec.gamma, beams=BEAMS,
                               baths=BATHS, dt=dt, nsteps=k0)
    s0 = {k: s[k] for k in tb.X + tb.V}
    t0 = s["t"]

    def run(beams=BEAMS, baths=BATHS, species=sp, gamma=spec.gamma):
        return oracle_mod.step_cooled(s0, w.charge, w.mass, species, tr, gamma, beams=beams,
                                      baths=baths, step_base=k0, t_start=t0, dt=dt, nsteps=SEG)

    def one(st, k):
        return oracle_mod.step_cooled(st, w.charge, w.mass, sp, tr, spec.gamma, beams=BEAMS,
                                      baths=BATHS, step_base=k0 + k, t_start=t0 + k * dt, dt=dt,
                                      nsteps=1)

    sc = oracle_mod.accel_scale(s0["x"], s0["y"], s0["z"], w.charge, w.mass, tr, t0)
    ref = run()
    kicked = tb.kicked_run(one, tb.nudge(s0), SEG, tb.kick(sc, tb.M1_REF, dt))
    return dict(run=run, one=one, s0=s0, sc=sc, ref=ref, kicked=kicked, sp=sp, dt=dt,
                beams=BEAMS, baths=BATHS, gamma=spec.gamma)


def _bars(c, r):
    return min(tb.ratio(r, c["ref"], c["kicked"], tb.X), tb.ratio(r, c["ref"], c["kicked"], tb.V))


def test_other_kick_realisation_stays_within_bars(cooled):
    c = cooled
    other = tb.kicked_run(c["one"], c["s0"], SEG, tb.kick(c["sc"], tb.M1_REF, c["dt"], seed=5))
    assert tb.ratio(other, c["ref"], c["kicked"], tb.X) < 1
    assert tb.ratio(other, c["ref"], c["kicked"], tb.V) < 1


@pytest.mark.parametrize("bath", [0, 1])
def test_wrong_bath_seed_is_caught(cooled, bath):
    c = cooled
    baths = [dict(b) for b in c["baths"]]
    baths[bath]["seed"] ^= 1
    assert _bars(c, c["run"](baths=baths)) >= 10


def test_swapped_species_are_caught(cooled):
    c = cooled
    assert _bars(c, c["run"](species=1 - c["sp"])) >= 10


@pytest.mark.parametrize("beam", [0, 1])
def test_beam_rate_off_by_a_thousandth_is_caught(cooled, beam):
    c = cooled
    beams = [dict(b) for b in c["beams"]]
    beams[beam]["gamma"] *= 1.001
    assert _bars(c, c["run"](beams=beams)) >= 10


def test_damping_rate_off_by_a_thousandth_is_caught(cooled):
    c = cooled
    assert _bars(c, c["run"](gamma=c["gamma"] * 1.001)) >= 10


@pytest.mark.parametrize("case", ["rod", "clusters"])
def test_changed_body_id_is_caught(oracle_mod, case):
    """Rigid bodies: the segment from step 170 of the GPU rigid test's runs; one
    ion taken out of its body, or a free ion put into one, moves the segment by
    far more than 10 bars; another kick realisation stays within them."""
    from tests.test_gpu_rigid import _clusters, _rod_and_cloud
    from tests.test_gpu_rigid import _trap as rigid_trap

    st, m, q, body = _rod_and_cloud() if case == "rod" else _clusters()
    tr = rigid_trap(oracle_mod)
    a, rg = oracle_mod.step_rigid(st, q, m, body, tr, 1e5, 0.0, li.DT, 170)
    s0 = {k: a[k] for k in tb.X + tb.V}
    t0 = a["t"]
    sc = oracle_mod.accel_bodies(s0["x"], s0["y"], s0["z"], q, m, body, tr, t0)[3]
    ref, kick_rigid, one, init = tb.rigid_segment(oracle_mod, s0, rg, q, m, body, tr, 1e5, t0,
                                                  li.DT)
    kicked = tb.kicked_run(one, init, SEG, tb.kick(sc, tb.M1_REF, li.DT), kick_rigid)
    other = tb.kicked_run(one, init, SEG, tb.kick(sc, tb.M1_REF, li.DT, seed=5), kick_rigid)
    assert tb.ratio(other, ref, kicked, tb.X) < 1 and tb.ratio(other, ref, kicked, tb.V) < 1
    members, free = np.nonzero(body >= 0)[0], np.nonzero(body < 0)[0]
    for i, new in ((members[0], -1), (members[4], -1), (free[0], body[members[0]])):
        b2 = body.copy()
        b2[i] = new
        r2, _ = oracle_mod.step_rigid(s0, q, m, b2, tr, 1e5, t0, li.DT, SEG)
        assert min(tb.ratio(r2, ref, kicked, tb.X), tb.ratio(r2, ref, kicked, tb.V)) >= 10, i

