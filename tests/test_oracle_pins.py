"""Pins of the oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper (or the textbook fact) it rests on.
A plausible slip in the oracle -- a dropped Coulomb or trap term, a flipped dc
or rf sign, a swapped pair index, a wrong damping placement or a wrong
constant -- fails at least one of them.
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

import lion_inputs as li
from tests import analytic

HERE = os.path.dirname(os.path.abspath(__file__))
CA = 40.0 * li.AMU
E = li.E_CHARGE


def _trap(oracle, q_x=0.3, a_x=-0.001, rf=True, dc=True):
    V0, U0 = oracle.voltages_for(q_x, a_x, CA, E, li.OMEGA, li.R0, li.Z0, li.KAPPA)
    return oracle.Trap(V0=V0 if rf else 0.0, Omega=li.OMEGA, U0=U0 if dc else 0.0, R0=li.R0,
                       Z0=li.Z0, kappa=li.KAPPA)


def _golden(name):
    rows = []
    with open(os.path.join(HERE, "golden", name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ----------------------------------------------------------------- constants

def test_constants_agree(oracle_mod):
    """Oracle, input generator and the 40-digit reference use the same SI values."""
    assert oracle_mod.E_CHARGE == li.E_CHARGE == analytic.E
    assert oracle_mod.AMU == li.AMU == analytic.AMU
    assert oracle_mod.EPS0 == analytic.EPS0
    assert oracle_mod.coulomb_constant() == pytest.approx(8.9875517923e9, rel=1e-10, abs=0)


# -------------------------------------------------------- brute force, N <= 4

@pytest.mark.parametrize("n,seed", [(2, 0), (3, 1), (4, 2)])
def test_accel_matches_40_digit_bruteforce(oracle_mod, n, seed):
    """Coulomb field (eq. fullPotential) + trap field (eq. field): the oracle's
    accel and scale agree with a 40-digit evaluation to a few ulp."""
    rng = np.random.default_rng(seed)
    x, y, z = rng.normal(0, 20e-6, (3, n))
    charge = rng.choice([-2.0, 1.0, 1.0, 3.0], n) * E
    mass = rng.uniform(10, 200, n) * li.AMU
    tr = _trap(oracle_mod)
    t = 1.234567e-7
    ax, ay, az = oracle_mod.accel(x, y, z, charge, mass, tr, t)
    sc = oracle_mod.accel_scale(x, y, z, charge, mass, tr, t)
    rx, ry, rz, rs = analytic.decimal_accel(x, y, z, charge, mass, tr.V0, tr.Omega, tr.U0, tr.R0,
                                            tr.Z0, tr.kappa, t)
    err = np.sqrt((ax - rx) ** 2 + (ay - ry) ** 2 + (az - rz) ** 2) / rs
    assert np.max(err) < 1e-15
    np.testing.assert_allclose(sc, rs, rtol=1e-14)


def test_ten_steps_match_40_digit_bruteforce(oracle_mod):
    """Damped velocity Verlet with Coulomb + dc trap (rf off) agrees with a
    40-digit integration of the same scheme over 10 steps."""
    rng = np.random.default_rng(7)
    n = 3
    st = {k: rng.normal(0, 20e-6, n) for k in ("x", "y", "z")}
    st.update({k: rng.normal(0, 1.0, n) for k in ("vx", "vy", "vz")})
    charge = np.array([1.0, 2.0, 1.0]) * E
    mass = np.array([40.0, 17.0, 88.0]) * li.AMU
    tr = _trap(oracle_mod, rf=False)
    out = oracle_mod.step(st, charge, mass, tr, 2e5, 0.0, li.DT, 10)
    ref = analytic.decimal_steps(st, charge, mass, tr.U0, tr.Z0, tr.kappa, 2e5, li.DT, 10)
    for p in ("x", "y", "z"):
        assert np.max(np.abs(out[p] - ref[p])) < 1e-13 * np.max(np.abs(ref[p]))
    for v in ("vx", "vy", "vz"):
        assert np.max(np.abs(out[v] - ref[v])) < 1e-12 * np.max(np.abs(ref[v]))
    assert out["t"] == 10 * li.DT


# ------------------------------------------------------- Newton's third law

def test_newton_third_law(oracle_mod):
    """Internal Coulomb forces cancel: |sum_i Q_i E_c,i| is rounding-sized."""
    w = li.random_cloud(64, seed=11, charge_e=np.random.default_rng(3).choice([1, 2, -1], 64))
    ex, ey, ez, c = oracle_mod.coulomb_field(w.x, w.y, w.z, w.charge)
    assert c == 0
    fx, fy, fz = w.charge * ex, w.charge * ey, w.charge * ez
    scale = np.sum(np.abs(w.charge) * np.sqrt(ex ** 2 + ey ** 2 + ez ** 2))
    assert abs(fx.sum()) < 1e-14 * scale
    assert abs(fy.sum()) < 1e-14 * scale
    assert abs(fz.sum()) < 1e-14 * scale


# ---------------------------------------------------------------- symmetries

def test_rotation_and_relabelling(oracle_mod):
    """A 180-degree turn about z maps a -> (-ax, -ay, az) exactly; relabelling
    ions permutes the accelerations (up to summation order)."""
    w = li.random_cloud(40, seed=5)
    tr = _trap(oracle_mod)
    t = 3.3e-8
    ax, ay, az = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, t)
    bx, by, bz = oracle_mod.accel(-w.x, -w.y, w.z, w.charge, w.mass, tr, t)
    assert np.array_equal(bx, -ax) and np.array_equal(by, -ay) and np.array_equal(bz, az)
    p = np.random.default_rng(1).permutation(40)
    cx, cy, cz = oracle_mod.accel(w.x[p], w.y[p], w.z[p], w.charge[p], w.mass[p], tr, t)
    sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, t)
    err = np.sqrt((cx - ax[p]) ** 2 + (cy - ay[p]) ** 2 + (cz - az[p]) ** 2) / sc[p]
    assert np.max(err) < 1e-15


def test_sampled_accel_equals_full(oracle_mod):
    """The sampled-target evaluation is the same definition: identical bits."""
    w = li.random_cloud(300, seed=12)
    tr = _trap(oracle_mod)
    ax, ay, az = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 1e-7)
    sc = oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 1e-7)
    idx = np.array([0, 5, 17, 299, 150])
    bx, by, bz, bs = oracle_mod.accel_at(w.x, w.y, w.z, w.charge, w.mass, tr, 1e-7, idx)
    assert np.array_equal(bx, ax[idx]) and np.array_equal(by, ay[idx])
    assert np.array_equal(bz, az[idx]) and np.array_equal(bs, sc[idx])


def test_coincident_pair_contributes_zero(oracle_mod):
    """Exactly coincident ions feel no mutual force (a select, not softening)."""
    x = np.array([0.0, 0.0, 10e-6])
    y = np.zeros(3)
    z = np.zeros(3)
    q = np.full(3, E)
    ex, ey, ez, c = oracle_mod.coulomb_field(x, y, z, q)
    assert c == 2
    k = oracle_mod.coulomb_constant()
    assert ex[0] == pytest.approx(-k * E / 1e-10, rel=1e-15, abs=0)
    assert ex[2] == pytest.approx(2 * k * E / 1e-10, rel=1e-15, abs=0)


# -------------------------------------------------- single-ion linear dynamics

@pytest.mark.parametrize("axis", ["x", "y", "z"])
def test_single_ion_matches_transfer_matrices(oracle_mod, axis):
    """Single ion, full rf + dc field, damping: the oracle's trajectory equals
    the product of independently written 2x2 step maps for x'' = k(t) x with
    k_x = (Q/M)(A_rf cos Omega t + A_dc), k_y = (Q/M)(-A_rf cos Omega t + A_dc),
    k_z = -2 (Q/M) A_dc (eq. field, confining dc reading)."""
    tr = _trap(oracle_mod)
    arf = tr.V0 / tr.R0 ** 2
    adc = tr.kappa * tr.U0 / tr.Z0 ** 2
    qm = E / CA
    kf = {"x": lambda t: qm * (arf * math.cos(tr.Omega * t) + adc),
          "y": lambda t: qm * (-arf * math.cos(tr.Omega * t) + adc),
          "z": lambda t: -2.0 * qm * adc}[axis]
    gamma = 3e4
    f = math.exp(-(gamma * li.DT) * 0.5)
    st = {k: np.zeros(1) for k in ("x", "y", "z", "vx", "vy", "vz")}
    st[axis][0] = 7e-6
    st["v" + axis][0] = 0.4
    nsteps = 400
    xs, vs = analytic.linear_trajectory(7e-6, 0.4, kf, f, li.DT, nsteps)
    cur = st
    t = 0.0
    for k in range(0, nsteps, 50):
        cur = oracle_mod.step(cur, [E], [CA], tr, gamma, t, li.DT, 50)
        t = cur["t"]
        assert abs(cur[axis][0] - xs[k + 50]) < 1e-12 * 7e-6
        assert abs(cur["v" + axis][0] - vs[k + 50]) < 1e-10 * 0.4
        others = [a for a in "xyz" if a != axis]
        assert all(cur[o][0] == 0.0 for o in others)


def test_secular_frequency_pseudopotential(oracle_mod):
    """Section 'Verifications', secular motion frequencies: the strongest Fourier
    component of a single ion's radial motion lies within 3 % of eq. (pseudopot)
    (the approximation itself is ~2 % low at q = 0.3), and within one FFT bin of
    the exact discrete Floquet value; the axial one matches the discrete
    harmonic frequency."""
    tr = _trap(oracle_mod)
    q, a = 0.3, -0.001
    nsteps = 1 << 15
    st = {k: np.zeros(1) for k in ("x", "y", "z", "vx", "vy", "vz")}
    st["x"][0] = 5e-6
    st["z"][0] = 5e-6
    xs, zs = [], []
    cur, t = st, 0.0
    # sample every 4 steps: Nyquist 9.6 MHz, far above the secular lines
    stride = 4
    for _ in range(nsteps // stride):
        cur = oracle_mod.step(cur, [E], [CA], tr, 0.0, t, li.DT, stride)
        t = cur["t"]
        xs.append(cur["x"][0])
        zs.append(cur["z"][0])
    fs = 1.0 / (stride * li.DT)
    freqs = np.fft.rfftfreq(len(xs), 1.0 / fs)
    bin_w = freqs[1]
    px = np.abs(np.fft.rfft(np.array(xs) * np.hanning(len(xs))))
    pz = np.abs(np.fft.rfft(np.array(zs) * np.hanning(len(zs))))
    sel = freqs < 1.5e6  # secular band, below the rf line at 3.85 MHz
    fx = freqs[sel][np.argmax(px[sel][1:]) + 1]
    fz = freqs[sel][np.argmax(pz[sel][1:]) + 1]
    f_pseudo = oracle_mod.pseudopotential_frequency(q, a, li.OMEGA) / (2 * math.pi)
    assert abs(fx - f_pseudo) / f_pseudo < 0.03
    arf = tr.V0 / tr.R0 ** 2
    adc = tr.kappa * tr.U0 / tr.Z0 ** 2
    qm = E / CA
    beta = analytic.floquet_beta(lambda tt: qm * (arf * math.cos(tr.Omega * tt) + adc),
                                 2 * math.pi / tr.Omega, 20)
    f_floquet = beta * li.OMEGA / 2 / (2 * math.pi)
    assert abs(fx - f_floquet) <= 1.01 * bin_w
    wz = math.sqrt(2 * qm * adc)
    f_disc = (2 / li.DT) * math.asin(wz * li.DT / 2) / (2 * math.pi)
    assert abs(fz - f_disc) <= 1.01 * bin_w
    # eq. (pseudopot) along z with q_z = 0, a_z = -2 a_x is the same frequency
    assert oracle_mod.pseudopotential_frequency(0.0, -2 * a, li.OMEGA) == pytest.approx(wz,
                                                                                          rel=1e-9, abs=0)


def test_paper_example_traps_are_consistent(oracle_mod):
    """The trap settings printed in the paper's examples (golden file): the
    Mathieu coefficients of eq. (Mathieuaq) predict, via eq. (pseudopot), the
    secular frequency that a single ion shows in the full field of eq. (field)
    within the 3 % the approximation allows at these q."""
    for name, V0, U0, R0, Z0, kappa, rf, qe, mu in _golden("paper_examples.txt"):
        V0, U0, R0, Z0, kappa, rf, qe, mu = map(float, (V0, U0, R0, Z0, kappa, rf, qe, mu))
        Om = 2 * math.pi * rf
        M, Q = mu * li.AMU, qe * E
        q, a = oracle_mod.mathieu_coefficients(V0, U0, M, Q, Om, R0, Z0, kappa)
        assert 0 < q < 0.9 and a < 0, name
        V0b, U0b = oracle_mod.voltages_for(q, a, M, Q, Om, R0, Z0, kappa)
        assert V0b == pytest.approx(V0, rel=1e-14, abs=0) and U0b == pytest.approx(U0, rel=1e-14, abs=0)
        tr = oracle_mod.Trap(V0=V0, Omega=Om, U0=U0, R0=R0, Z0=Z0, kappa=kappa)
        dt = 1.0 / rf / 20
        stride, nsamp = 4, 4096
        cur = {k: np.zeros(1) for k in ("x", "y", "z", "vx", "vy", "vz")}
        cur["x"][0] = 3e-6
        xs, t = [], 0.0
        for _ in range(nsamp):
            cur = oracle_mod.step(cur, [Q], [M], tr, 0.0, t, dt, stride)
            t = cur["t"]
            xs.append(cur["x"][0])
        freqs = np.fft.rfftfreq(nsamp, stride * dt)
        px = np.abs(np.fft.rfft(np.array(xs) * np.hanning(nsamp)))
        sel = freqs < 0.4 * rf
        f_sim = freqs[sel][np.argmax(px[sel][1:]) + 1]
        f_ps = oracle_mod.pseudopotential_frequency(q, a, Om) / (2 * math.pi)
        # the paper quotes the approximation as good to ~1 % up to q = 0.4; beyond
        # that (the rigid-body example has q ~ 0.55) allow the larger error it has
        tol = 0.03 if q <= 0.4 else 0.10
        assert abs(f_sim - f_ps) / f_ps < tol + freqs[1] / f_ps, name
        qm = Q / M
        arf, adc = V0 / R0 ** 2, kappa * U0 / Z0 ** 2
        beta = analytic.floquet_beta(lambda tt: qm * (arf * math.cos(Om * tt) + adc), 1 / rf, 20)
        assert abs(f_sim - beta * rf / 2) <= 1.01 * freqs[1], name


# -------------------------------------------------------------- Kohn theorem

def test_centre_of_mass_follows_single_ion(oracle_mod):
    """Linear trap forces + cancelling internal forces: the centre of mass of a
    single-species cloud follows the one-ion trajectory started from the centre
    of mass (full rf field and damping)."""
    w = li.random_cloud(16, seed=21, sigma=30e-6)
    tr = _trap(oracle_mod)
    st = w.state()
    com = {k: np.array([np.mean(st[k])]) for k in st}
    run = oracle_mod.step(st, w.charge, w.mass, tr, 1e5, 0.0, li.DT, 2000)
    one = oracle_mod.step(com, [E], [CA], tr, 1e5, 0.0, li.DT, 2000)
    for k in ("x", "y", "z"):
        amp = np.max(np.abs(st[k]))
        assert abs(np.mean(run[k]) - one[k][0]) < 1e-9 * amp, k


# ------------------------------------------------------------ chain spacings

def _relax_chain(oracle_mod, n, tr, nsteps=30000):
    st = {k: np.zeros(n) for k in ("x", "y", "z", "vx", "vy", "vz")}
    st["z"] = np.linspace(-1.0, 1.0, n) * 12e-6 * max(n - 1, 1) ** 0.7
    return oracle_mod.step(st, np.full(n, E), np.full(n, CA), tr, 1e6, 0.0, li.DT, nsteps)


def _length_scale(tr):
    wz2 = 2 * E * tr.kappa * tr.U0 / (CA * tr.Z0 ** 2)
    return (E * E / (4 * math.pi * analytic.EPS0 * CA * wz2)) ** (1 / 3)


def test_two_ion_spacing_closed_form(oracle_mod):
    """d = (e^2 / (2 pi eps0 M omega_z^2))^(1/3) for two damped ions on the axis."""
    tr = _trap(oracle_mod, rf=False)
    out = _relax_chain(oracle_mod, 2, tr)
    wz2 = 2 * E * tr.kappa * tr.U0 / (CA * tr.Z0 ** 2)
    d = (E * E / (2 * math.pi * analytic.EPS0 * CA * wz2)) ** (1 / 3)
    assert out["z"][1] - out["z"][0] == pytest.approx(d, rel=1e-11, abs=0)
    assert out["z"][0] + out["z"][1] == pytest.approx(0.0, abs=1e-20)


def test_three_ion_spacing_closed_form(oracle_mod):
    """Three ions: 0 and +-(5/4)^(1/3) l."""
    tr = _trap(oracle_mod, rf=True)  # on the axis the rf field vanishes identically
    out = _relax_chain(oracle_mod, 3, tr)
    lsc = _length_scale(tr)
    z = np.sort(out["z"])
    assert z[2] == pytest.approx((5 / 4) ** (1 / 3) * lsc, rel=1e-11, abs=0)
    assert z[0] == pytest.approx(-(5 / 4) ** (1 / 3) * lsc, rel=1e-11, abs=0)
    assert abs(z[1]) < 1e-12 * lsc


@pytest.mark.parametrize("n", [4, 6, 9])
def test_chain_matches_newton_root(oracle_mod, n):
    """N-ion chains relax to the independent root of the axial force balance."""
    tr = _trap(oracle_mod, rf=False)
    out = _relax_chain(oracle_mod, n, tr, nsteps=60000)
    u = np.sort(out["z"]) / _length_scale(tr)
    np.testing.assert_allclose(u, analytic.chain_equilibrium(n), atol=1e-9)


def test_chain_minimum_spacing_matches_paper_fit(oracle_mod):
    """Section 'Verifications', equilibrium separation: z_min / l within 3 % of
    the printed fit 2.018 / N^0.559 (golden file) for 3 <= N <= 10."""
    coef, expo, tol, nmin, nmax = map(float, _golden("zmin_fit.txt")[0])
    tr = _trap(oracle_mod, rf=False)
    for n in range(int(nmin), int(nmax) + 1):
        out = _relax_chain(oracle_mod, n, tr, nsteps=40000)
        zmin = np.min(np.diff(np.sort(out["z"]))) / _length_scale(tr)
        fit = coef / n ** expo
        assert abs(zmin - fit) / fit < tol, n


def test_breathing_mode_is_sqrt3_omega_z(oracle_mod):
    """Axial modes of a chain in a harmonic well: the centre-of-mass mode is at
    omega_z and the breathing mode at sqrt(3) omega_z for any N (textbook).
    Checked via the linearised force of the relaxed 5-ion chain."""
    tr = _trap(oracle_mod, rf=False)
    n = 5
    out = _relax_chain(oracle_mod, n, tr)
    z0 = out["z"].copy()
    h = 1e-11
    H = np.zeros((n, n))
    zeros = np.zeros(n)
    for j in range(n):
        zp, zm = z0.copy(), z0.copy()
        zp[j] += h
        zm[j] -= h
        ap = oracle_mod.accel(zeros, zeros, zp, np.full(n, E), np.full(n, CA), tr, 0.0)[2]
        am = oracle_mod.accel(zeros, zeros, zm, np.full(n, E), np.full(n, CA), tr, 0.0)[2]
        H[:, j] = -(ap - am) / (2 * h)
    w = np.sqrt(np.sort(np.linalg.eigvalsh(0.5 * (H + H.T))))
    wz = math.sqrt(2 * E * tr.kappa * tr.U0 / (CA * tr.Z0 ** 2))
    assert w[0] == pytest.approx(wz, rel=1e-5, abs=0)
    assert w[1] == pytest.approx(math.sqrt(3) * wz, rel=1e-5, abs=0)


# ---------------------------------------------------- damping and energies

def test_laser_cooling_free_particle(oracle_mod):
    """Section 'Verifications', cooling mechanisms: with no fields a free ion's
    velocity decays as exp(-gamma t) (tau = 1 us), exactly for this scheme, and
    the position follows the matching geometric sum."""
    tr = oracle_mod.Trap()
    gamma = 1e6
    st = {k: np.zeros(1) for k in ("x", "y", "z", "vx", "vy", "vz")}
    st["vx"][0], st["vy"][0], st["vz"][0] = 3.0, -1.0, 0.5
    out = oracle_mod.step(st, [E], [CA], tr, gamma, 0.0, li.DT, 1000)
    decay = math.exp(-gamma * 1000 * li.DT)
    assert out["vx"][0] == pytest.approx(3.0 * decay, rel=1e-12, abs=0)
    assert out["vy"][0] == pytest.approx(-1.0 * decay, rel=1e-12, abs=0)
    f = math.exp(-gamma * li.DT / 2)
    xs = li.DT * 3.0 * f * (1 - f ** 2000) / (1 - f ** 2)
    assert out["x"][0] == pytest.approx(xs, rel=1e-12, abs=0)


def test_harmonic_shadow_energy(oracle_mod):
    """Single ion on the axis, rf off, no damping: v^2 + w^2 (1 - w^2 dt^2/4) z^2
    is an exact invariant of velocity Verlet for a harmonic force."""
    tr = _trap(oracle_mod, rf=False)
    wz2 = 2 * E * tr.kappa * tr.U0 / (CA * tr.Z0 ** 2)
    st = {k: np.zeros(1) for k in ("x", "y", "z", "vx", "vy", "vz")}
    st["z"][0], st["vz"][0] = 4e-6, 1.5
    inv0 = st["vz"][0] ** 2 + wz2 * (1 - wz2 * li.DT ** 2 / 4) * st["z"][0] ** 2
    out = oracle_mod.step(st, [E], [CA], tr, 0.0, 0.0, li.DT, 100000)
    inv = out["vz"][0] ** 2 + wz2 * (1 - wz2 * li.DT ** 2 / 4) * out["z"][0] ** 2
    assert inv == pytest.approx(inv0, rel=1e-11, abs=0)


def test_energy_conserved_on_axis_chain(oracle_mod):
    """Rf off, no damping, ions on the axis (radial forces vanish identically):
    kinetic + Coulomb + dc energy shows bounded O(dt^2) wobble and no drift."""
    tr = _trap(oracle_mod, rf=False)
    n = 5
    st = {k: np.zeros(n) for k in ("x", "y", "z", "vx", "vy", "vz")}
    st["z"] = np.linspace(-40e-6, 40e-6, n)
    st["vz"] = np.array([0.5, -1.0, 0.2, 0.8, -0.3])
    q, m = np.full(n, E), np.full(n, CA)
    es = []
    cur, t = st, 0.0
    for _ in range(40):
        cur = oracle_mod.step(cur, q, m, tr, 0.0, t, li.DT, 500)
        t = cur["t"]
        es.append(sum(oracle_mod.energy(cur, q, m, tr)))
    es = np.array(es)
    e0 = sum(oracle_mod.energy(st, q, m, tr))
    assert np.max(np.abs(es - e0)) / abs(e0) < 1e-4
    assert abs(np.mean(es[:10]) - np.mean(es[-10:])) / abs(e0) < 1e-6


def test_coulomb_explosion_conserves_energy_and_momentum(oracle_mod):
    """No trap, no damping: total energy and total momentum are conserved."""
    w = li.random_cloud(12, seed=9, sigma=20e-6, temperature=1e-3)
    tr = oracle_mod.Trap()
    st = w.state()
    e0 = sum(oracle_mod.energy(st, w.charge, w.mass, tr))
    out = oracle_mod.step(st, w.charge, w.mass, tr, 0.0, 0.0, li.DT / 4, 4000)
    e1 = sum(oracle_mod.energy(out, w.charge, w.mass, tr))
    assert e1 == pytest.approx(e0, rel=1e-6, abs=0)
    for v in ("vx", "vy", "vz"):
        p0, p1 = np.sum(w.mass * st[v]), np.sum(w.mass * out[v])
        assert abs(p1 - p0) < 1e-12 * np.sum(w.mass * np.abs(out[v]))


def test_energy_gradient_is_minus_force(oracle_mod):
    """The Coulomb + dc energies are potentials of the oracle's static field:
    central differences of the energy equal -Q_i (E_c + E_dc) on every axis."""
    w = li.random_cloud(6, seed=4)
    tr = _trap(oracle_mod, rf=False)
    st = w.state()
    ax, ay, az = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    h = 1e-10
    for i in (0, 3):
        for p, a in (("x", ax), ("y", ay), ("z", az)):
            sp, sm = dict(st), dict(st)
            sp[p] = st[p].copy()
            sm[p] = st[p].copy()
            sp[p][i] += h
            sm[p][i] -= h
            ep = sum(oracle_mod.energy(sp, w.charge, w.mass, tr)[1:])
            em = sum(oracle_mod.energy(sm, w.charge, w.mass, tr)[1:])
            force = -(ep - em) / (2 * h)
            assert force == pytest.approx(w.mass[i] * a[i], rel=1e-5, abs=0)


# ------------------------------------------------------------------- batches

def test_batch_equals_independent_traps(oracle_mod):
    """Batched traps do not interact: each trap evolves as if alone."""
    w = li.batch512(n_traps=5, n_min=2, n_max=12, seed=8, nsteps=0)
    traps = []
    for ts in w.traps:
        V0, U0 = oracle_mod.voltages_for(ts.q_x, ts.a_x, CA, E, ts.omega, ts.r0, ts.z0, ts.kappa)
        traps.append(oracle_mod.Trap(V0=V0, Omega=ts.omega, U0=U0, R0=ts.r0, Z0=ts.z0,
                                     kappa=ts.kappa))
    st = w.state()
    g = np.array([ts.gamma for ts in w.traps])
    dt = np.array([ts.dt for ts in w.traps])
    t0 = np.zeros(len(traps))
    out = oracle_mod.step_batch(w.offsets, st, w.charge, w.mass, traps, g, t0, dt, 30)
    for k in range(len(traps)):
        o, e = w.offsets[k], w.offsets[k + 1]
        sub = {kk: st[kk][o:e] for kk in st}
        one = oracle_mod.step(sub, w.charge[o:e], w.mass[o:e], traps[k], g[k], 0.0, dt[k], 30)
        for kk in ("x", "y", "z", "vx", "vy", "vz", "ax"):
            assert np.array_equal(out[kk][o:e], one[kk])


# ------------------------------------------------------------ rigid bodies

def test_body_exclusion_matches_40_digit_bruteforce(oracle_mod):
    """Pairs inside a rigid body are left out (section 'Charged rigid body'):
    4 ions, ions 0 and 2 bound together, against a 40-digit evaluation."""
    rng = np.random.default_rng(17)
    x, y, z = rng.normal(0, 20e-6, (3, 4))
    charge = np.array([1.0, 2.0, 1.0, -1.0]) * E
    mass = rng.uniform(10, 200, 4) * li.AMU
    body = np.array([0, -1, 0, -1], dtype=np.int32)
    tr = _trap(oracle_mod)
    ax, ay, az, sc = oracle_mod.accel_bodies(x, y, z, charge, mass, body, tr, 2e-8)
    rx, ry, rz, rs = analytic.decimal_accel(x, y, z, charge, mass, tr.V0, tr.Omega, tr.U0, tr.R0,
                                            tr.Z0, tr.kappa, 2e-8, body=body)
    err = np.sqrt((ax - rx) ** 2 + (ay - ry) ** 2 + (az - rz) ** 2) / rs
    assert np.max(err) < 1e-15
    np.testing.assert_allclose(sc, rs, rtol=1e-14)


def test_body_exclusion_special_cases(oracle_mod):
    """All ions free: identical to accel; one body holding every ion: only the
    trap field acts; internal forces of the rest still cancel pairwise."""
    w = li.random_cloud(50, seed=23)
    tr = _trap(oracle_mod)
    free = np.full(50, -1, dtype=np.int32)
    ax, ay, az, sc = oracle_mod.accel_bodies(w.x, w.y, w.z, w.charge, w.mass, free, tr, 1e-8)
    bx, by, bz = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 1e-8)
    assert np.array_equal(ax, bx) and np.array_equal(ay, by) and np.array_equal(az, bz)
    assert np.array_equal(sc, oracle_mod.accel_scale(w.x, w.y, w.z, w.charge, w.mass, tr, 1e-8))
    one = np.zeros(50, dtype=np.int32)
    cx, cy, cz, _ = oracle_mod.accel_bodies(w.x, w.y, w.z, w.charge, w.mass, one, tr, 1e-8)
    nq = oracle_mod.Trap()  # no field: no force at all
    dx, dy, dz, _ = oracle_mod.accel_bodies(w.x, w.y, w.z, w.charge, w.mass, one, nq, 1e-8)
    assert np.all(dx == 0) and np.all(dy == 0) and np.all(dz == 0)
    ex, ey, ez = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 1e-8)
    fx, fy, fz, _ = oracle_mod.coulomb_field(w.x, w.y, w.z, w.charge)
    qm = w.charge / w.mass
    np.testing.assert_allclose(cx, ex - qm * fx, rtol=1e-9, atol=1e-9 * np.max(np.abs(ex)))
    # bodies of 10 ions: the net internal force on each body vanishes with the
    # excluded pairs, and the total over all ions still cancels (Newton)
    groups = (np.arange(50) // 10).astype(np.int32)
    nofield = oracle_mod.Trap()
    gx, gy, gz, gs = oracle_mod.accel_bodies(w.x, w.y, w.z, w.charge, w.mass, groups, nofield, 0.0)
    f = w.mass * gx
    assert abs(f.sum()) < 1e-13 * np.sum(np.abs(f))


def test_sampled_body_accel_equals_full(oracle_mod):
    """The sampled-target body evaluation is the same definition: identical bits."""
    w = li.random_cloud(200, seed=31)
    body = (np.arange(200) // 25 - 3).astype(np.int32)  # ids -3.. -> free for negatives
    body[body < 0] = -1
    tr = _trap(oracle_mod)
    ax, ay, az, sc = oracle_mod.accel_bodies(w.x, w.y, w.z, w.charge, w.mass, body, tr, 3e-8)
    idx = np.array([0, 74, 75, 199, 120])
    bx, by, bz, bs = oracle_mod.accel_bodies_at(w.x, w.y, w.z, w.charge, w.mass, body, tr, 3e-8,
                                                idx)
    assert np.array_equal(bx, ax[idx]) and np.array_equal(by, ay[idx])
    assert np.array_equal(bz, az[idx]) and np.array_equal(bs, sc[idx])


# ------------------------------------------------- cooling beams and baths

def test_philox_known_answers(oracle_mod):
    """The bath's random numbers: Philox4x32-10 against its published vectors."""
    for row in _golden("philox_kat.txt"):
        w = [int(v, 16) for v in row]
        assert oracle_mod.philox4x32_10(w[0:4], w[4:6]) == tuple(w[6:10])


def test_bath_normals_are_standard(oracle_mod):
    """Box-Muller of Philox outputs: zero mean, unit variance, uncorrelated."""
    z = np.array([oracle_mod.normals3(12345, i, 7, 1, 0) for i in range(20000)])
    assert np.all(np.abs(z.mean(0)) < 4 / np.sqrt(20000))
    assert np.all(np.abs(z.var(0) - 1) < 4 * np.sqrt(2 / 20000))
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(3))) < 4 / np.sqrt(20000)
    # different half-step, step, bath or seed: a different draw
    base = oracle_mod.normals3(1, 5, 9, 0, 0)
    for args in ((1, 5, 9, 0, 1), (1, 5, 10, 0, 0), (1, 5, 9, 1, 0), (2, 5, 9, 0, 0),
                 (1, 6, 9, 0, 0)):
        assert not np.array_equal(base, oracle_mod.normals3(*args))


def test_cooled_step_without_cooling_is_plain_step(oracle_mod):
    w = li.random_cloud(30, seed=51)
    tr = _trap(oracle_mod)
    a = oracle_mod.step(w.state(), w.charge, w.mass, tr, 1e5, 0.0, li.DT, 40)
    b = oracle_mod.step_cooled(w.state(), w.charge, w.mass, np.zeros(30), tr, 1e5, dt=li.DT,
                               nsteps=40)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(a[k], b[k])


def test_single_beam_cooling_free_ions(oracle_mod):
    """Section 'Verifications', cooling mechanisms: free, non-interacting ions
    cooled along one random axis (tau = 1 us): the velocity along the beam
    decays as exp(-t/tau), the perpendicular components are untouched, and ions
    of another species are not cooled at all."""
    rng = np.random.default_rng(3)
    k = rng.normal(size=3)
    k /= np.linalg.norm(k)
    n = 6
    st = {p: np.zeros(n) for p in ("x", "y", "z")}
    v = rng.normal(0, 2.0, (3, n))
    st.update(vx=v[0], vy=v[1], vz=v[2])
    species = np.array([0, 0, 0, 1, 1, 0], dtype=np.int32)
    q0 = np.zeros(n)  # neutral: no Coulomb force
    m = np.full(n, CA)
    beam = dict(k=k, gamma=1e6, species=0)
    out = oracle_mod.step_cooled(st, q0, m, species, oracle_mod.Trap(), 0.0, beams=[beam],
                                 dt=li.DT, nsteps=800)
    vin = np.stack([st["vx"], st["vy"], st["vz"]])
    vout = np.stack([out["vx"], out["vy"], out["vz"]])
    decay = math.exp(-1e6 * 800 * li.DT)
    for i in range(n):
        par_in, par_out = k @ vin[:, i], k @ vout[:, i]
        perp_in, perp_out = vin[:, i] - par_in * k, vout[:, i] - par_out * k
        if species[i] == 0:
            # every half-step rounds each velocity component to ~u |v|; on the
            # decayed parallel part these add up like a random walk over the
            # 1600 half-steps (~40 u |v|): bound 10x that
            assert par_out == pytest.approx(par_in * decay, rel=1e-11,
                                            abs=1e-13 * np.max(np.abs(vin[:, i])))
        else:
            assert np.array_equal(vout[:, i], vin[:, i])
        assert np.max(np.abs(perp_out - perp_in)) < 1e-14 * np.max(np.abs(vin[:, i]))


def test_langevin_baths_follow_newtons_law_of_cooling(oracle_mod):
    """Section 'Verifications', cooling mechanisms: groups of free,
    non-interacting ions, each coupled to its own bath (T_j, c_j), reach
    3 k_B T = M <v^2> along T(t) = T_j + (T0 - T_j) exp(-2 t / c_j)."""
    groups = [(1e-3, 10e-6), (5e-3, 30e-6), (0.2e-3, 5e-6)]
    per = 1000
    n = per * len(groups)
    T0 = 2e-3
    m = np.full(n, CA)
    rng = np.random.default_rng(9)
    s0 = np.sqrt(li.K_B * T0 / CA)
    st = {p: np.zeros(n) for p in ("x", "y", "z")}
    v = rng.normal(0, s0, (3, n))
    st.update(vx=v[0], vy=v[1], vz=v[2])
    species = np.repeat(np.arange(len(groups)), per).astype(np.int32)
    baths = [dict(temperature=T, tau=tau, seed=1000 + g, species=g)
             for g, (T, tau) in enumerate(groups)]
    dt = 1e-7
    cur, done = st, 0
    temps0 = [CA * np.mean(v[:, species == g] ** 2) / li.K_B for g in range(len(groups))]
    for chunk in (50, 100, 150):
        cur = oracle_mod.step_cooled(cur, np.zeros(n), m, species, oracle_mod.Trap(), 0.0,
                                     baths=baths, step_base=done, t_start=done * dt, dt=dt,
                                     nsteps=chunk)
        done += chunk
        t = done * dt
        vv = np.stack([cur["vx"], cur["vy"], cur["vz"]])
        for g, (T, tau) in enumerate(groups):
            meas = CA * np.mean(vv[:, species == g] ** 2) / li.K_B
            pred = T + (temps0[g] - T) * math.exp(-2 * t / tau)
            sigma = pred * math.sqrt(2 / (3 * per))
            assert abs(meas - pred) < 4 * sigma, (g, t, meas, pred)


def test_bath_draws_follow_run_wide_ion_numbering(oracle_mod):
    """A trap inside a batch draws its bath kicks as ions ion_base.. of the run:
    for neutral ions (no coupling) the last five ions of a ten-ion run equal a
    five-ion run with ion_base = 5, and differ from one with ion_base = 0."""
    n = 10
    rng = np.random.default_rng(21)
    st = {p: rng.normal(0, 1e-5, n) for p in ("x", "y", "z")}
    st.update({p: rng.normal(0, 0.5, n) for p in ("vx", "vy", "vz")})
    m = np.full(n, CA)
    sp = np.zeros(n, dtype=np.int32)
    bath = [dict(temperature=1e-3, tau=5e-6, seed=77)]
    tr = _trap(oracle_mod)
    full = oracle_mod.step_cooled(st, np.zeros(n), m, sp, tr, 1e5, baths=bath, dt=li.DT,
                                  nsteps=25, step_base=3)
    tail = {k: v[5:] for k, v in st.items()}
    part = oracle_mod.step_cooled(tail, np.zeros(5), m[5:], sp[5:], tr, 1e5, baths=bath,
                                  dt=li.DT, nsteps=25, step_base=3, ion_base=5)
    wrong = oracle_mod.step_cooled(tail, np.zeros(5), m[5:], sp[5:], tr, 1e5, baths=bath,
                                   dt=li.DT, nsteps=25, step_base=3, ion_base=0)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.array_equal(full[k][5:], part[k])
        assert not np.array_equal(full[k][5:], wrong[k])


def test_time_average_of_damped_free_ion_closed_form(oracle_mod):
    """timeAvg over windows of W steps: for a free ion under isotropic damping
    the velocity after step s is v0 r^s with r = exp(-gamma dt) (each step
    applies two exact half-step factors), so the mean over the window of steps
    a .. a + W - 1 is the geometric sum (v0 / W) r^a (1 - r^W) / (1 - r).
    Averaging started at step 3: windows close at steps 23 and 43."""
    gamma, dt, W, origin = 1e6, li.DT, 20, 3
    st = {k: np.array([v]) for k, v in
          (("x", 0.0), ("y", 0.0), ("z", 0.0), ("vx", 2.5), ("vy", -1.0), ("vz", 0.25))}
    samples, t = [], 0.0
    for _ in range(60):
        st = oracle_mod.step(st, [li.E_CHARGE], [li.REF_MASS], oracle_mod.Trap(), gamma, t, dt, 1)
        t = st["t"]
        samples.append([st["vx"][0], st["vy"][0], st["vz"][0]])
    ends, means = oracle_mod.time_average(np.array(samples), 1, origin, W)
    assert list(ends) == [23, 43]
    r = math.exp(-gamma * dt)
    for end, mean in zip(ends, means):
        a = end - W + 1
        geo = r ** a * (1 - r ** W) / (1 - r) / W
        for v0, m in zip((2.5, -1.0, 0.25), mean):
            assert m == pytest.approx(v0 * geo, rel=1e-12, abs=0)


def test_time_average_window_alignment(oracle_mod):
    """Samples equal to their step number average to the window's mid-step
    exactly; windows reaching before the first sample are skipped; constant
    samples average to themselves bit for bit."""
    steps = np.arange(10, 31, dtype=np.float64)  # samples of steps 10 .. 30
    ends, means = oracle_mod.time_average(steps, 10, 0, 4)
    assert list(ends) == [16, 20, 24, 28]  # the window 9 .. 12 starts before step 10
    assert np.array_equal(means[:, 0], (ends - 1.5).astype(np.float64))
    c = np.full((12, 3), 0.1)
    ends, means = oracle_mod.time_average(c, 1, 0, 3)
    assert list(ends) == [3, 6, 9, 12]
    assert np.all(np.abs(means - 0.1) <= 2 * np.finfo(float).eps * 0.1)


# ------------------------------------------------------------ rigid bodies

def _rod(n=9, spacing=2.5e-6):
    """The paper's rod: ions on the z axis, 2.5 um apart, centred at 0."""
    z = (np.arange(n) - (n - 1) / 2) * spacing
    return np.zeros(n), np.zeros(n), z


def _rigid_cloud(n_free, seed, sigma=100e-6, rod_at=(0.0, 0.0, 0.0)):
    rng = np.random.default_rng(seed)
    rx, ry, rz = _rod()
    x = np.concatenate([rng.normal(0, sigma, n_free), rx + rod_at[0]])
    y = np.concatenate([rng.normal(0, sigma, n_free), ry + rod_at[1]])
    z = np.concatenate([rng.normal(0, sigma, n_free), rz + rod_at[2]])
    n = x.size
    v = rng.normal(0, 1.0, (3, n))
    body = np.concatenate([np.full(n_free, -1), np.zeros(9)]).astype(np.int32)
    st = dict(x=x, y=y, z=z, vx=v[0], vy=v[1], vz=v[2])
    return st, np.full(n, CA), np.full(n, li.E_CHARGE), body


def test_rigid_singleton_bodies_are_free_ions(oracle_mod):
    """A body of one ion has no moments of inertia and nothing to exclude: it
    moves exactly as a free ion (to the rounding of F/M = (m a)/m)."""
    w = li.random_cloud(12, seed=71, sigma=40e-6)
    tr = _trap(oracle_mod)
    a = oracle_mod.step(w.state(), w.charge, w.mass, tr, 1e5, 0.0, li.DT, 300)
    b, _ = oracle_mod.step_rigid(w.state(), w.charge, w.mass, np.arange(12), tr, 1e5, 0.0, li.DT,
                                 300)
    ext = np.max(np.abs(w.x))
    for k in ("x", "y", "z"):
        assert np.max(np.abs(a[k] - b[k])) < 1e-12 * ext, k


def test_rigid_body_com_follows_single_ion(oracle_mod):
    """Kohn for a body: the trap field is linear and every member has the same
    Q/M, so the summed force is Q_tot E(R) and a lone body's centre of mass
    follows the one-ion trajectory exactly, whatever its rotation does."""
    st, m, q, body = _rigid_cloud(0, seed=5)
    for k in ("x", "y", "z"):
        st[k] = st[k] + {"x": 7e-6, "y": -4e-6, "z": 11e-6}[k]
    tr = _trap(oracle_mod)
    out, rg = oracle_mod.step_rigid(st, q, m, body, tr, 1e5, 0.0, li.DT, 2000)
    setup = oracle_mod.rigid_setup(st, m, body)
    one = {"x": setup["R"][0, :1].copy(), "y": setup["R"][0, 1:2].copy(),
           "z": setup["R"][0, 2:3].copy(), "vx": setup["V"][0, :1].copy(),
           "vy": setup["V"][0, 1:2].copy(), "vz": setup["V"][0, 2:3].copy()}
    ref = oracle_mod.step(one, [li.E_CHARGE], [CA], tr, 1e5, 0.0, li.DT, 2000)
    for c, k in enumerate("xyz"):
        assert abs(rg["R"][0, c] - ref[k][0]) < 1e-10 * 11e-6, k


def _rod_spinning(omega0=2e5):
    """Rod on z spinning about x at omega0: member velocities omega x d."""
    x, y, z = _rod()
    n = x.size
    w = np.array([omega0, 0.0, 0.0])
    v = np.cross(w, np.stack([x, y, z], 1))
    st = dict(x=x, y=y, z=z, vx=v[:, 0].copy(), vy=v[:, 1].copy(), vz=v[:, 2].copy())
    return st, np.full(n, CA), np.zeros(n), np.zeros(n, dtype=np.int32)


def test_rigid_rod_spin_is_uniform_rotation(oracle_mod):
    """Torque-free rod spinning about a perpendicular axis: the exact motion is
    a uniform rotation about that axis.  The scheme is second order (error
    falls 4x when dt halves) and the member velocities are omega x d."""
    omega0 = 2e5
    st, m, q, body = _rod_spinning(omega0)
    T = 1.0 / omega0  # one radian
    errs = []
    for nsteps in (100, 200):
        dt = T / nsteps
        out, _ = oracle_mod.step_rigid(st, q, m, body, oracle_mod.Trap(), 0.0, 0.0, dt, nsteps)
        ang = omega0 * T
        ey = -np.sin(ang) * st["z"]
        ez = np.cos(ang) * st["z"]
        errs.append(max(np.max(np.abs(out["y"] - ey)), np.max(np.abs(out["z"] - ez)),
                        np.max(np.abs(out["x"]))))
        d = np.stack([out["x"], out["y"], out["z"]], 1)
        v = np.stack([out["vx"], out["vy"], out["vz"]], 1)
        assert np.allclose(v, np.cross([omega0, 0, 0], d), rtol=0, atol=1e-9 * omega0 * 1e-5)
    ext = np.max(np.abs(st["z"]))
    assert errs[0] < 1e-4 * ext
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


def _free_body_reference(A0, inv_i, L_space, T):
    """Free rigid body from Euler's equations in the body frame, integrated by
    scipy (DOP853): d pi/dt = pi x (I^-1 pi), dA/dt = A [I^-1 pi]_x."""
    from scipy.integrate import solve_ivp

    def rhs(_, y):
        A = y[:9].reshape(3, 3)
        pi = y[9:]
        w = inv_i * pi
        wx = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        return np.concatenate([(A @ wx).ravel(), np.cross(pi, w)])

    y0 = np.concatenate([A0.ravel(), A0.T @ L_space])
    sol = solve_ivp(rhs, (0, T), y0, method="DOP853", rtol=1e-13, atol=1e-15 * np.abs(y0).max())
    return sol.y[:9, -1].reshape(3, 3)


def test_rigid_asymmetric_top_converges_to_euler_equations(oracle_mod):
    """A lone asymmetric body (5 ions), no field: member positions after a time
    T agree with an independent high-order solution of Euler's equations, with
    second-order convergence; the space-frame angular momentum is untouched."""
    rng = np.random.default_rng(12)
    n = 5
    p = rng.normal(0, 3e-6, (n, 3))
    v = rng.normal(0, 1.0, (n, 3))
    st = dict(x=p[:, 0], y=p[:, 1], z=p[:, 2], vx=v[:, 0], vy=v[:, 1], vz=v[:, 2])
    m = CA * np.array([1.0, 1.3, 0.7, 2.0, 1.1])
    body = np.zeros(n, dtype=np.int32)
    setup = oracle_mod.rigid_setup(st, m, body)
    A0 = oracle_mod.quaternion_matrix(setup["q"][0])
    wmax = np.linalg.norm(A0 @ (setup["inv_i"][0] * (A0.T @ setup["L"][0])))
    T = 2.0 / wmax
    A_ref = _free_body_reference(A0, setup["inv_i"][0], setup["L"][0], T)
    R = setup["R"][0]
    ref = R + T * setup["V"][0] + setup["dbody"] @ A_ref.T
    errs = []
    for nsteps in (200, 400):
        out, rg = oracle_mod.step_rigid(st, np.zeros(n), m, body, oracle_mod.Trap(), 0.0, 0.0,
                                        T / nsteps, nsteps)
        got = np.stack([out["x"], out["y"], out["z"]], 1)
        errs.append(np.max(np.abs(got - ref)))
        assert np.array_equal(rg["L"][0], setup["L"][0])
    assert errs[0] < 1e-3 * np.max(np.abs(setup["dbody"]))
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


def test_rigid_spin_down_under_damping(oracle_mod):
    """Isotropic damping scales every member velocity, hence V and L, by
    exp(-gamma dt) per step: a torque-free spinning rod loses its angular
    momentum as exp(-gamma t)."""
    st, m, q, body = _rod_spinning()
    setup = oracle_mod.rigid_setup(st, m, body)
    gamma, nsteps = 3e5, 500
    _, rg = oracle_mod.step_rigid(st, q, m, body, oracle_mod.Trap(), gamma, 0.0, li.DT, nsteps)
    decay = math.exp(-gamma * nsteps * li.DT)
    assert rg["L"][0, 0] == pytest.approx(setup["L"][0, 0] * decay, rel=1e-12, abs=0)


def test_rigid_coulomb_explosion_conserves_momenta(oracle_mod):
    """No trap, no damping: a rod, a 4-ion body and 25 free ions repel.  Pair
    forces are central and pairs inside a body are left out, so total momentum
    and total angular momentum (orbital + body spin) are conserved to rounding;
    the energy to O(dt^2)."""
    rng = np.random.default_rng(33)
    st, m, q, body = _rigid_cloud(25, seed=34, sigma=15e-6)
    extra = rng.normal(0, 2e-6, (4, 3)) + [20e-6, -10e-6, 5e-6]
    for c, k in enumerate("xyz"):
        st[k] = np.concatenate([st[k], extra[:, c]])
    for k in ("vx", "vy", "vz"):
        st[k] = np.concatenate([st[k], rng.normal(0, 1.0, 4)])
    m = np.concatenate([m, np.full(4, CA)])
    q = np.concatenate([q, np.full(4, li.E_CHARGE)])
    body = np.concatenate([body, np.full(4, 7)]).astype(np.int32)
    free = body < 0
    ke = oracle_mod.coulomb_constant()

    def invariants(s, rg):
        r = np.stack([s["x"], s["y"], s["z"]], 1)
        v = np.stack([s["vx"], s["vy"], s["vz"]], 1)
        P = (m[free, None] * v[free]).sum(0) + (rg["M"][:, None] * rg["V"]).sum(0)
        J = (m[free, None] * np.cross(r[free], v[free])).sum(0) + \
            (rg["M"][:, None] * np.cross(rg["R"], rg["V"])).sum(0) + rg["L"].sum(0)
        E = 0.5 * np.sum(m[:, None] * v * v)
        for i in range(r.shape[0]):
            for j in range(i + 1, r.shape[0]):
                if body[i] >= 0 and body[i] == body[j]:
                    continue
                E += ke * q[i] * q[j] / np.linalg.norm(r[i] - r[j])
        pscale = np.sum(m[:, None] * np.abs(v))
        jscale = np.sum(m * np.linalg.norm(r, axis=1) * np.linalg.norm(v, axis=1))
        return P, J, E, pscale, jscale

    setup = oracle_mod.rigid_setup(st, m, body)
    s0 = dict(st, vx=setup["vx"], vy=setup["vy"], vz=setup["vz"])
    P0, J0, E0, ps, js = invariants(s0, setup)
    out, rg = oracle_mod.step_rigid(st, q, m, body, oracle_mod.Trap(), 0.0, 0.0, 2e-9, 400)
    P1, J1, E1, _, _ = invariants(out, rg)
    assert np.max(np.abs(P1 - P0)) < 1e-13 * ps
    assert np.max(np.abs(J1 - J0)) < 1e-12 * js
    assert abs(E1 - E0) < 1e-5 * abs(E0)


def test_rigid_members_keep_their_distances(oracle_mod):
    """The paper's rod among 30 ions in the trap, 2000 steps: distances between
    members are preserved to rounding."""
    st, m, q, body = _rigid_cloud(30, seed=2)
    out, _ = oracle_mod.step_rigid(st, q, m, body, _trap(oracle_mod), 1e5, 0.0, li.DT, 2000)
    r0 = np.stack([st["x"], st["y"], st["z"]], 1)[body == 0]
    r1 = np.stack([out["x"], out["y"], out["z"]], 1)[body == 0]
    d0 = np.linalg.norm(r0[:, None] - r0[None], axis=2)
    d1 = np.linalg.norm(r1[:, None] - r1[None], axis=2)
    assert np.max(np.abs(d1 - d0)) < 1e-12 * np.max(d0)


# ------------------------------------------------------------ pseudopotential trap

def _pseudo_trap(oracle, q_x=0.3, a_x=-0.001):
    V0, U0 = oracle.voltages_for(q_x, a_x, CA, E, li.OMEGA, li.R0, li.Z0, li.KAPPA)
    return oracle.Trap(V0=V0, Omega=li.OMEGA, U0=U0, R0=li.R0, Z0=li.Z0, kappa=li.KAPPA,
                       pseudo=True)


@pytest.mark.parametrize("mass_u", [40.0, 17.0])
def test_pseudo_trap_single_ion_is_harmonic(oracle_mod, mass_u):
    """In the pseudopotential trap ("Electric fields and confinement":
    linearPseudoPT) one ion is a harmonic oscillator on each axis with the
    frequency of eq. (pseudopot), using that ion's own Mathieu coefficients
    (eq. (Mathieuaq) scales with Q/M).  The oracle's run equals the exact
    velocity-Verlet transfer matrix of that oscillator."""
    tr = _pseudo_trap(oracle_mod)
    m = mass_u * li.AMU
    q_x, a_x = oracle_mod.mathieu_coefficients(tr.V0, tr.U0, m, E, tr.Omega, tr.R0, tr.Z0,
                                               tr.kappa)
    w_r = oracle_mod.pseudopotential_frequency(q_x, a_x, tr.Omega)
    w_z = oracle_mod.pseudopotential_frequency(0.0, -2 * a_x, tr.Omega)
    dt, n = li.DT, 3000
    st = {"x": np.array([3e-6]), "y": np.array([-2e-6]), "z": np.array([5e-6]),
          "vx": np.array([0.4]), "vy": np.array([0.7]), "vz": np.array([-0.3])}
    out = oracle_mod.step(st, [E], [m], tr, 0.0, 0.0, dt, n)
    for p, v, w in (("x", "vx", w_r), ("y", "vy", w_r), ("z", "vz", w_z)):
        c = 1 - (w * dt) ** 2 / 2
        T = np.array([[c, dt], [-w * w * dt * (1 - (w * dt) ** 2 / 4), c]])
        ref = np.linalg.matrix_power(T, n) @ np.array([st[p][0], st[v][0]])
        amp = math.hypot(st[p][0], st[v][0] / w)
        assert abs(out[p][0] - ref[0]) < 1e-11 * amp, p
        assert abs(out[v][0] - ref[1]) < 1e-11 * amp * w, v


def test_pseudo_energy_gradient_is_minus_force(oracle_mod):
    """The pseudopotential trap's static energy (dc + radial pseudopotential)
    plus the Coulomb energy is the potential of the oracle's force, for two
    species."""
    w = li.random_cloud(6, seed=14, light_fraction=0.5)
    tr = _pseudo_trap(oracle_mod)
    st = w.state()
    ax, ay, az = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    h = 1e-10
    for i in range(6):
        for p, a in (("x", ax), ("y", ay), ("z", az)):
            sp, sm = dict(st), dict(st)
            sp[p] = st[p].copy()
            sm[p] = st[p].copy()
            sp[p][i] += h
            sm[p][i] -= h
            ep = sum(oracle_mod.energy(sp, w.charge, w.mass, tr)[1:])
            em = sum(oracle_mod.energy(sm, w.charge, w.mass, tr)[1:])
            force = -(ep - em) / (2 * h)
            assert force == pytest.approx(w.mass[i] * a[i], rel=1e-5, abs=0)


def test_pseudo_trap_is_time_independent(oracle_mod):
    """The pseudopotential field does not depend on t."""
    w = li.random_cloud(10, seed=15, light_fraction=0.3)
    tr = _pseudo_trap(oracle_mod)
    a0 = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    a1 = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 3.3e-8)
    for c0, c1 in zip(a0, a1):
        assert np.array_equal(c0, c1)


# ------------------------------------------------------------------ minimisation

def _force_unit(tr):
    """M omega_z^2 l: the natural force scale of a chain (N)."""
    wz2 = 2 * E * tr.kappa * tr.U0 / (CA * tr.Z0 ** 2)
    return CA * wz2 * _length_scale(tr)


def _min_start(n, seed, spread=1.0):
    """Ions roughly along the axis with off-axis scatter, at rest."""
    rng = np.random.default_rng(seed)
    st = {k: np.zeros(n) for k in ("vx", "vy", "vz")}
    st["z"] = np.linspace(-1.0, 1.0, n) * 12e-6 * max(n - 1, 1) ** 0.7 + rng.normal(0, 1e-6, n)
    st["x"] = rng.normal(0, spread * 1e-6, n)
    st["y"] = rng.normal(0, spread * 1e-6, n)
    return st


@pytest.mark.parametrize("n", [2, 3, 5, 10])
def test_minimised_chains_match_newton_roots(oracle_mod, n):
    """Section 'Equilibrium separation': minimising eq. (fullPotential) in the
    pseudopotential trap from a scattered start gives the linear chain; its
    positions equal the independent Newton roots of the axial force balance,
    and for 3 <= N <= 10 the minimum spacing is within 3 % of the printed
    z_min fit (golden file)."""
    tr = _pseudo_trap(oracle_mod)
    l, fu = _length_scale(tr), _force_unit(tr)
    out = oracle_mod.minimize(_min_start(n, seed=n), np.full(n, E), np.full(n, CA), tr,
                              dt=2e-8, dmax=1e-6, ftol=1e-10 * fu, max_iter=200000)
    assert out["fmax"] <= 1e-10 * fu
    assert np.max(np.abs(out["x"])) < 1e-9 * l and np.max(np.abs(out["y"])) < 1e-9 * l
    u = np.sort(out["z"]) / l
    assert np.max(np.abs(u - analytic.chain_equilibrium(n))) < 1e-8
    if n >= 3:
        coef, expo, tol, _, _ = map(float, _golden("zmin_fit.txt")[0])
        fit = coef / n ** expo
        assert abs(np.min(np.diff(u)) - fit) / fit < tol


def test_minimised_crystal_is_a_local_minimum(oracle_mod):
    """A 30-ion, two-species cloud minimised in the pseudopotential trap: the
    force is below tolerance, the energy fell, and the energy rises along 20
    random small displacements (second-order test of a minimum)."""
    w = li.random_cloud(30, seed=17, sigma=20e-6, light_fraction=0.3)
    tr = _pseudo_trap(oracle_mod)
    fu = _force_unit(tr)
    st = w.state()
    for k in ("vx", "vy", "vz"):
        st[k] = np.zeros(30)
    out = oracle_mod.minimize(st, w.charge, w.mass, tr, dt=2e-8, dmax=1e-6, ftol=1e-9 * fu,
                              max_iter=200000)
    assert out["fmax"] <= 1e-9 * fu

    def pot(s):
        return sum(oracle_mod.energy(s, w.charge, w.mass, tr)[1:])

    e_min = pot(out)
    assert e_min < pot(st)
    rng = np.random.default_rng(3)
    l = _length_scale(tr)
    for _ in range(20):
        d = rng.normal(size=(3, 30)) * 1e-3 * l
        s2 = dict(out, x=out["x"] + d[0], y=out["y"] + d[1], z=out["z"] + d[2])
        assert pot(s2) > e_min


def test_minimiser_step_cap_and_projection(oracle_mod):
    """One iteration from a far-off start: every ion moves at most dmax; a
    velocity pointing against the force is dropped (only dt a remains)."""
    w = li.random_cloud(8, seed=18, sigma=200e-6)
    tr = _pseudo_trap(oracle_mod)
    st = w.state()
    ax, ay, az = oracle_mod.accel(w.x, w.y, w.z, w.charge, w.mass, tr, 0.0)
    st.update(vx=-ax * 1e-7, vy=-ay * 1e-7, vz=-az * 1e-7)  # v . F < 0
    dmax = 1e-7
    out = oracle_mod.minimize(st, w.charge, w.mass, tr, dt=1e-8, dmax=dmax, ftol=0.0,
                              max_iter=1)
    assert out["iterations"] == 1
    step = np.sqrt((out["x"] - w.x) ** 2 + (out["y"] - w.y) ** 2 + (out["z"] - w.z) ** 2)
    assert np.all(step <= dmax * (1 + 1e-12))
    v = np.stack([out["vx"], out["vy"], out["vz"]])
    a = np.stack([ax, ay, az])
    small = 1e-16 * np.linalg.norm(a, axis=0) <= dmax  # moves dt^2 |a| below the cap
    assert np.any(small) and not np.all(small)
    assert np.allclose(v[:, small], 1e-8 * a[:, small], rtol=1e-15, atol=0)
    capped = ~small
    assert np.allclose(step[capped], dmax, rtol=1e-12, atol=0)


# ------------------------------------------------------------------ normal modes

def _pseudo_freqs(oracle_mod, tr, mass):
    q_x, a_x = oracle_mod.mathieu_coefficients(tr.V0, tr.U0, mass, E, tr.Omega, tr.R0, tr.Z0,
                                               tr.kappa)
    return (oracle_mod.pseudopotential_frequency(q_x, a_x, tr.Omega),
            oracle_mod.pseudopotential_frequency(0.0, -2 * a_x, tr.Omega))


@pytest.mark.parametrize("mass_u", [40.0, 17.0])
def test_normal_modes_of_one_ion(oracle_mod, mass_u):
    """One ion: the three modes are the trap's eq. (pseudopot) frequencies."""
    tr = _pseudo_trap(oracle_mod)
    m = mass_u * li.AMU
    w_r, w_z = _pseudo_freqs(oracle_mod, tr, m)
    w2, _ = oracle_mod.normal_modes([1e-6], [-2e-6], [3e-6], [E], [m], tr)
    assert np.allclose(np.sort(w2), np.sort([w_r ** 2, w_r ** 2, w_z ** 2]), rtol=1e-12, atol=0)


def _james_chain_modes(n, alpha):
    """Axial and radial mode eigenvalues (units of omega_z^2) of an n-ion chain
    from the dimensionless equilibrium u (independent 1-D computation):
    axial A_ii = 1 + sum_p 2/|u_i-u_p|^3, A_ij = -2/|u_i-u_j|^3;
    radial B_ii = alpha - sum_p 1/|u_i-u_p|^3, B_ij = 1/|u_i-u_j|^3."""
    u = analytic.chain_equilibrium(n)
    d = np.abs(u[:, None] - u[None, :])
    np.fill_diagonal(d, np.inf)
    c = 1.0 / d ** 3
    A = -2 * c
    np.fill_diagonal(A, 1 + 2 * c.sum(1))
    B = c.copy()
    np.fill_diagonal(B, alpha - c.sum(1))
    return np.linalg.eigvalsh(A), np.linalg.eigvalsh(B)


@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_normal_modes_of_minimised_chains(oracle_mod, n):
    """Section 'Normal modes of motion': the modes of an n-ion chain minimised
    in 3D equal the axial and radial spectra computed from the 1-D equilibrium;
    the COM mode is omega_z, the breathing mode sqrt(3) omega_z, the two-ion
    rocking mode sqrt(omega_r^2 - omega_z^2), and the 3-ion third axial mode
    sqrt(29/5) omega_z."""
    tr = _pseudo_trap(oracle_mod)
    w_r, w_z = _pseudo_freqs(oracle_mod, tr, CA)
    fu = _force_unit(tr)
    out = oracle_mod.minimize(_min_start(n, seed=30 + n), np.full(n, E), np.full(n, CA), tr,
                              dt=2e-8, dmax=1e-6, ftol=1e-12 * fu, max_iter=400000)
    w2, _ = oracle_mod.normal_modes(out["x"], out["y"], out["z"], np.full(n, E),
                                    np.full(n, CA), tr)
    ax, rad = _james_chain_modes(n, (w_r / w_z) ** 2)
    ref = np.sort(np.concatenate([ax, rad, rad])) * w_z ** 2
    assert np.allclose(np.sort(w2), ref, rtol=1e-8, atol=0)
    got = np.sqrt(np.sort(w2)) / w_z
    assert np.min(np.abs(got - 1.0)) < 1e-8
    if n >= 2:
        assert np.min(np.abs(got - math.sqrt(3))) < 1e-8
    if n == 2:
        assert np.min(np.abs(got - math.sqrt((w_r / w_z) ** 2 - 1))) < 1e-8
    if n == 3:
        assert np.min(np.abs(got - math.sqrt(29 / 5))) < 1e-8


def test_normal_modes_kohn_and_trace(oracle_mod):
    """Any one-species configuration: the trace of the mass-weighted Hessian is
    n (2 omega_r^2 + omega_z^2) (the Coulomb blocks are traceless, the Laplacian
    of 1/r vanishing); at a minimised 3D crystal the spectrum contains the
    three centre-of-mass frequencies exactly."""
    tr = _pseudo_trap(oracle_mod)
    w_r, w_z = _pseudo_freqs(oracle_mod, tr, CA)
    w = li.random_cloud(25, seed=31, sigma=20e-6)
    D = oracle_mod.hessian(w.x, w.y, w.z, w.charge, w.mass, tr)
    assert np.trace(D) == pytest.approx(25 * (2 * w_r ** 2 + w_z ** 2), rel=1e-10, abs=0)
    st = w.state()
    for k in ("vx", "vy", "vz"):
        st[k] = np.zeros(25)
    out = oracle_mod.minimize(st, w.charge, w.mass, tr, dt=2e-8, dmax=1e-6,
                              ftol=1e-11 * _force_unit(tr), max_iter=400000)
    w2, _ = oracle_mod.normal_modes(out["x"], out["y"], out["z"], w.charge, w.mass, tr)
    for target in (w_r ** 2, w_z ** 2):
        assert np.min(np.abs(w2 - target)) < 1e-8 * target
    assert np.sum(np.abs(w2 - w_r ** 2) < 1e-8 * w_r ** 2) >= 2  # x and y COM modes


def test_hessian_is_minus_force_derivative(oracle_mod):
    """D = -sqrt(M_i/M_j) d a_i / d x_j, by central differences of the
    oracle's acceleration (two species, 5 ions)."""
    w = li.random_cloud(5, seed=32, sigma=20e-6, light_fraction=0.4)
    tr = _pseudo_trap(oracle_mod)
    D = oracle_mod.hessian(w.x, w.y, w.z, w.charge, w.mass, tr)
    pos = np.stack([w.x, w.y, w.z], 1)
    h = 1e-10
    for j in range(5):
        for b in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[j, b] += h
            pm[j, b] -= h
            ap = np.stack(oracle_mod.accel(pp[:, 0], pp[:, 1], pp[:, 2], w.charge, w.mass, tr, 0.0), 1)
            am = np.stack(oracle_mod.accel(pm[:, 0], pm[:, 1], pm[:, 2], w.charge, w.mass, tr, 0.0), 1)
            da = (ap - am) / (2 * h)
            col = -(da * np.sqrt(w.mass / w.mass[j])[:, None]).ravel()
            scale = np.max(np.abs(D))
            assert np.max(np.abs(D[:, 3 * j + b] - col)) < 1e-5 * scale, (j, b)
