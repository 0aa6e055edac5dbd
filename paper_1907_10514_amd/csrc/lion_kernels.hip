// HIP kernels for gfx950 (CDNA4): all-pairs Coulomb field, linear Paul trap
// field and damped velocity-Verlet update of trapped ions.
//
// Physics (paper, "Dynamics of trapped ions" eq. (field) and eq.
// (fullPotential); "Implementation details": unscreened pair sum, nve
// integration; "Cooling the motion of ions": viscous laser-cooling force):
//   S_i   = sum_{j != i} q_j (r_i - r_j) / |r_i - r_j|^3     (q_j = Q_j / e)
//   a_i   = (Q_i/M_i) [ k_e e S_i + A_rf cos(Omega t)(x, -y, 0) + A_dc (x, y, -2z) ]
//   step  v <- f v; v <- v + h a; x <- x + dt v; a <- a(x, t+dt); v <- f (v + h a)
//
// Layout of the single-trap step (one trap, any N):
//   pair kernel   grid (ceil(N / (256 I)), J): lane = I target ions held in
//                 registers, a wave walks one slice of the sources.  Source
//                 positions are wave-uniform, so they arrive through scalar
//                 loads straight into SGPRs and feed every lane without LDS
//                 traffic; each slice writes one partial sum per target.
//   update kernel per ion: sums the J partials in slice order (deterministic,
//                 no atomics), adds the trap field at t_{k+1}, applies the
//                 second half kick and damping and, inside a chunk, the first
//                 half of the next step (damping, half kick, drift).
// Batched traps: one workgroup per trap keeps the trap's source stream in LDS
// and runs many steps in one launch with workgroup barriers only.
//
// Pair arithmetic:
//   FP64  d = x_j - x_i; r2 = |d|^2; y0 = v_rsq_f64(r2) (~2^-24 relative);
//         q y^3 is formed with one folded Newton correction,
//         q r^-3 ~ q y0^3 (5/2 - 3/2 r2 y0^2), relative error ~7.5 e0^2 < 1e-13.
//   FP32  float-float positions (hi + lo, scaled by 2^20/m) give d with ~2 ulp
//         relative error even for close pairs of far-off-centre ions; r^-3 from
//         v_rsq_f32; sums in FP32 over short runs flushed to FP64, or Kahan.
#include <hip/hip_runtime.h>
#include <type_traits>
#include <math.h>

#include "lion_internal.h"

namespace lion {
namespace {

constexpr double kKeE = kElementaryCharge / (4.0 * kPi * kEps0);  // k_e e (V m)

// ------------------------------------------------------------------ pair terms

// One FP64 pair term, accumulated into (sx, sy, sz).  p = {x_j, y_j, z_j, 1.5 q_j}.
__device__ __forceinline__ void pair_f64(const double4 p, double xi, double yi, double zi,
                                         double& sx, double& sy, double& sz) {
    const double dx = p.x - xi, dy = p.y - yi, dz = p.z - zi;
    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, kR2FloorF64)));
    const double y = __builtin_amdgcn_rsq(r2);
    const double a = y * y;
    const double g = fma(r2, a, -5.0 / 3.0);  // (r2 y^2 - 5/3)
    const double w = (a * y) * p.w * g;       // 1.5 q y^3 (r2 y^2 - 5/3) = -q r^-3
    sx = fma(w, dx, sx);
    sy = fma(w, dy, sy);
    sz = fma(w, dz, sz);
}

// As pair_f64 for a source of unit weight: adds y^3 (r2 y^2 - 5/3) d, which
// times 1.5 q_j is the term of pair_f64 (the caller scales the sums).
__device__ __forceinline__ void pair_f64_unit(const double4 p, double xi, double yi, double zi,
                                              double& sx, double& sy, double& sz) {
    const double dx = p.x - xi, dy = p.y - yi, dz = p.z - zi;
    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, kR2FloorF64)));
    const double y = __builtin_amdgcn_rsq(r2);
    const double a = y * y;
    const double g = fma(r2, a, -5.0 / 3.0);
    const double w = (a * y) * g;
    sx = fma(w, dx, sx);
    sy = fma(w, dy, sy);
    sz = fma(w, dz, sz);
}

// Target-side float-float position.
struct FF {
    float xh, yh, zh, xl, yl, zl;
};

// One FP32 pair term on float-float positions; returns the three products.
// UNIT: the source weight -q is left out (the caller scales the sums).
template <bool UNIT = false>
__device__ __forceinline__ void pair_f32_terms(const MixedSrc& q, const FF& t, float& tx,
                                               float& ty, float& tz) {
    const float dx = (q.xh - t.xh) + (q.xl - t.xl);
    const float dy = (q.yh - t.yh) + (q.yl - t.yl);
    const float dz = (q.zh - t.zh) + (q.zl - t.zl);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, q.r2floor)));
    const float y = __builtin_amdgcn_rsqf(r2);
    const float w = UNIT ? y * (y * y) : (q.nq * y) * (y * y);  // -q r^-3 (r^-3 with UNIT)
    tx = w * dx;
    ty = w * dy;
    tz = w * dz;
}

// As pair_f32 for a source of unit weight (r^-3 d; the caller scales by -q).
__device__ __forceinline__ void pair_f32_unit(const MixedSrc& q, const FF& t, float& sx,
                                              float& sy, float& sz) {
    const float dx = (q.xh - t.xh) + (q.xl - t.xl);
    const float dy = (q.yh - t.yh) + (q.yl - t.yl);
    const float dz = (q.zh - t.zh) + (q.zl - t.zl);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, q.r2floor)));
    const float y = __builtin_amdgcn_rsqf(r2);
    const float w = y * (y * y);
    sx = fmaf(w, dx, sx);
    sy = fmaf(w, dy, sy);
    sz = fmaf(w, dz, sz);
}

__device__ __forceinline__ void pair_f32(const MixedSrc& q, const FF& t, float& sx, float& sy,
                                         float& sz) {
    const float dx = (q.xh - t.xh) + (q.xl - t.xl);
    const float dy = (q.yh - t.yh) + (q.yl - t.yl);
    const float dz = (q.zh - t.zh) + (q.zl - t.zl);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, q.r2floor)));
    const float y = __builtin_amdgcn_rsqf(r2);
    const float w = (q.nq * y) * (y * y);
    sx = fmaf(w, dx, sx);
    sy = fmaf(w, dy, sy);
    sz = fmaf(w, dz, sz);
}

// As pair_f64 / pair_f32, with the term dropped when source and target share a body.
__device__ __forceinline__ void pair_f64_masked(const double4 p, double xi, double yi,
                                                double zi, int ci, int cj, double& sx,
                                                double& sy, double& sz) {
    const double dx = p.x - xi, dy = p.y - yi, dz = p.z - zi;
    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, kR2FloorF64)));
    const double y = __builtin_amdgcn_rsq(r2);
    const double a = y * y;
    const double g = fma(r2, a, -5.0 / 3.0);
    const double w = (ci == cj) ? 0.0 : (a * y) * p.w * g;
    sx = fma(w, dx, sx);
    sy = fma(w, dy, sy);
    sz = fma(w, dz, sz);
}

// Kahan-compensated FP32 accumulation of one term.
__device__ __forceinline__ void kahan_add(float term, float& s, float& c) {
    const float y = term - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Rigid-body exclusion.  code[i] is ion i's body id (>= 0) or a negative
// number unique to the ion, so code[i] == code[j] (i != j) exactly when both
// ions belong to one body.  gmin/gmax give, per group of 16 consecutive ions,
// the range of body ids >= 0 present (gmin > gmax when there are none); a
// 16-source group whose range misses the targets' range needs no per-pair test.
struct BodyMask {
    const int32_t* __restrict__ code;
    const int32_t* __restrict__ gmin;
    const int32_t* __restrict__ gmax;
};

// Body-id range of the 64*I targets starting at base0 (a multiple of 64).
template <int I>
__device__ __forceinline__ void target_body_range(const BodyMask& bm, int64_t base0, int& lo,
                                                  int& hi) {
    lo = 0x7fffffff;
    hi = -1;
    for (int g = 0; g < 4 * I; ++g) {
        lo = min(lo, bm.gmin[base0 / 16 + g]);
        hi = max(hi, bm.gmax[base0 / 16 + g]);
    }
}

__device__ __forceinline__ bool group_may_share_body(const BodyMask& bm, int j16, int lo,
                                                     int hi) {
    return bm.code && bm.gmin[j16] <= hi && bm.gmax[j16] >= lo;
}

__device__ __forceinline__ FF split_ff(double x, double y, double z) {
    FF r;
    const double xs = x * kMixedScale, ys = y * kMixedScale, zs = z * kMixedScale;
    r.xh = (float)xs;
    r.yh = (float)ys;
    r.zh = (float)zs;
    r.xl = (float)(xs - (double)r.xh);
    r.yl = (float)(ys - (double)r.yh);
    r.zl = (float)(zs - (double)r.zh);
    return r;
}

__device__ __forceinline__ MixedSrc make_src(double x, double y, double z, double qe) {
    const FF f = split_ff(x, y, z);
    MixedSrc m;
    m.xh = f.xh;
    m.yh = f.yh;
    m.zh = f.zh;
    m.nq = (float)(-qe);
    m.xl = f.xl;
    m.yl = f.yl;
    m.zl = f.zl;
    m.r2floor = kR2FloorF32;
    return m;
}

// --------------------------------------------------------- trap field

// c = cos(Omega t) of the step's time (unused by the pseudopotential trap).
__device__ __forceinline__ void trap_accel_c(const TrapDev& T, double c, double qm, double x,
                                             double y, double z, double Sx, double Sy,
                                             double Sz, double& ax, double& ay, double& az) {
#pragma clang fp contract(off)
    if (T.ps != 0.0) {
        // pseudopotential trap: static radial field -(Q/M) A_rf^2/(2 Omega^2) (x, y, 0)
        const double k = qm * T.ps;
        const double ex = T.a_dc * x - k * x;
        const double ey = T.a_dc * y - k * y;
        const double ez = -2.0 * T.a_dc * z;
        ax = qm * (kKeE * Sx + ex);
        ay = qm * (kKeE * Sy + ey);
        az = qm * (kKeE * Sz + ez);
        return;
    }
    const double ex = T.a_rf * c * x + T.a_dc * x;
    const double ey = -T.a_rf * c * y + T.a_dc * y;
    const double ez = -2.0 * T.a_dc * z;
    ax = qm * (kKeE * Sx + ex);
    ay = qm * (kKeE * Sy + ey);
    az = qm * (kKeE * Sz + ez);
}

__device__ __forceinline__ void trap_accel(const TrapDev& T, double t, double qm, double x,
                                           double y, double z, double Sx, double Sy, double Sz,
                                           double& ax, double& ay, double& az) {
    trap_accel_c(T, T.ps != 0.0 ? 0.0 : cos(T.omega * t), qm, x, y, z, Sx, Sy, Sz, ax, ay, az);
}

// ------------------------------------------------------------ cooling

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32
// multiplications with the round key bumped by the Weyl constants.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Three standard normals for (seed, ion, step, bath, half-step): Box-Muller of
// the four Philox words taken as uniforms (r + 1/2) 2^-32.
__device__ __forceinline__ void bath_normals(uint64_t seed, int64_t ion, int64_t step, int bath,
                                             int half, double& z0, double& z1, double& z2) {
#pragma clang fp contract(off)
    uint32_t c[4] = {(uint32_t)ion, (uint32_t)((uint64_t)step & 0xffffffffu),
                     (uint32_t)((uint64_t)step >> 32), ((uint32_t)bath << 8) | (uint32_t)half};
    philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    const double s32 = 1.0 / 4294967296.0;
    const double u1 = ((double)c[0] + 0.5) * s32, u2 = ((double)c[1] + 0.5) * s32;
    const double u3 = ((double)c[2] + 0.5) * s32, u4 = ((double)c[3] + 0.5) * s32;
    const double r1 = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
    z0 = r1 * cos(2.0 * kPi * u2);
    z1 = r1 * sin(2.0 * kPi * u2);
    z2 = r2 * cos(2.0 * kPi * u4);
}

// The cooling and averaging switches, read once per launch: they cannot change
// during one, and re-reading them after every barrier of an in-kernel step
// loop costs more than the step's arithmetic for small traps.
struct CoolRef {
    const CoolDev* C;
    int nb, nt, W;
    int64_t origin;
};

// X = false: a kernel built with beams, baths and time averages compiled out
// (all switches constant zero), launched while none of them is on.
template <bool X>
__device__ __forceinline__ CoolRef cool_switches(const CoolDev* __restrict__ C);

__device__ __forceinline__ CoolRef load_cool(const CoolDev* __restrict__ C) {
    CoolRef r;
    r.C = C;
    r.nb = C ? C->nbeams : 0;
    r.nt = C ? C->nbaths : 0;
    r.W = C ? C->avg_window : 0;
    r.origin = C ? C->avg_origin : 0;
    return r;
}

template <bool X>
__device__ __forceinline__ CoolRef cool_switches(const CoolDev* __restrict__ C) {
    if constexpr (X) {
        return load_cool(C);
    } else {
        return CoolRef{nullptr, 0, 0, 0, 0};
    }
}

// Velocity half-step: isotropic damping f, then beams, then baths (index order).
__device__ __forceinline__ void velocity_half(const CoolRef& R, int64_t ion,
                                              int32_t species, double mass, double f,
                                              int64_t step, int half, double& u, double& v,
                                              double& w) {
#pragma clang fp contract(off)
    u = f * u;
    v = f * v;
    w = f * w;
    const int nb = R.nb, nt = R.nt;
    if (nb == 0 && nt == 0) return;
    const CoolDev* __restrict__ C = R.C;
    for (int b = 0; b < nb; ++b) {
        const BeamDev B = C->beams[b];
        if (!B.on || (B.species >= 0 && B.species != species)) continue;
        const double d = (1.0 - B.f) * (B.kx * u + B.ky * v + B.kz * w);
        u = u - d * B.kx;
        v = v - d * B.ky;
        w = w - d * B.kz;
    }
    for (int c = 0; c < nt; ++c) {
        const BathDev T = C->baths[c];
        if (!T.on || (T.species >= 0 && T.species != species)) continue;
        const double sig = sqrt(T.kt / mass * T.omc2);
        double z0, z1, z2;
        bath_normals(T.seed, ion, step, c, half, z0, z1, z2);
        u = T.c1 * u + sig * z0;
        v = T.c1 * v + sig * z1;
        w = T.c1 * w + sig * z2;
    }
}

// Velocity time average over windows of W steps: the velocity at the end of
// each step is added to the open window's sums; the step that closes a window
// publishes sums / W and restarts the sums.  `step` is the run-wide number of
// the step just completed.
__device__ __forceinline__ void time_average(const CoolRef& R, int64_t i,
                                             int64_t n_pad, int64_t step, double* __restrict__ acc,
                                             double* __restrict__ avg, double u, double v,
                                             double w) {
#pragma clang fp contract(off)
    const int W = R.W;
    if (W <= 0) return;
    const double sx = acc[i] + u, sy = acc[n_pad + i] + v, sz = acc[2 * n_pad + i] + w;
    if ((step - R.origin) % W == 0) {
        avg[i] = sx / (double)W;
        avg[n_pad + i] = sy / (double)W;
        avg[2 * n_pad + i] = sz / (double)W;
        acc[i] = 0.0;
        acc[n_pad + i] = 0.0;
        acc[2 * n_pad + i] = 0.0;
    } else {
        acc[i] = sx;
        acc[n_pad + i] = sy;
        acc[2 * n_pad + i] = sz;
    }
}

// First half of a step: velocity half-step (damping, beams, baths), half kick,
// drift.  `step` numbers steps from 1 over the whole run.
__device__ __forceinline__ void half_step_drift(const TrapDev& T, const CoolRef& C,
                                                int64_t ion, int32_t species, double mass,
                                                int64_t step, double& x, double& y, double& z,
                                                double& vx, double& vy, double& vz, double ax,
                                                double ay, double az) {
#pragma clang fp contract(off)
    velocity_half(C, ion, species, mass, T.f, step, 0, vx, vy, vz);
    vx = vx + T.h * ax;
    vy = vy + T.h * ay;
    vz = vz + T.h * az;
    x = x + T.dt * vx;
    y = y + T.dt * vy;
    z = z + T.dt * vz;
}

// Second half of a step: half kick with the new acceleration, velocity half-step.
__device__ __forceinline__ void end_kick(const TrapDev& T, const CoolRef& C,
                                         int64_t ion, int32_t species, double mass, int64_t step,
                                         double& vx, double& vy, double& vz, double ax, double ay,
                                         double az) {
#pragma clang fp contract(off)
    vx = vx + T.h * ax;
    vy = vy + T.h * ay;
    vz = vz + T.h * az;
    velocity_half(C, ion, species, mass, T.f, step, 1, vx, vy, vz);
}

// ------------------------------------------------------------------ kernels

template <bool X>
__global__ __launch_bounds__(256) void k_drift(double4* __restrict__ src,
                                               MixedSrc* __restrict__ srcm,
                                               double* __restrict__ vx, double* __restrict__ vy,
                                               double* __restrict__ vz,
                                               const double* __restrict__ ax,
                                               const double* __restrict__ ay,
                                               const double* __restrict__ az,
                                               const double* __restrict__ qe,
                                               const double* __restrict__ mass,
                                               const int32_t* __restrict__ species,
                                               const TrapDev* __restrict__ traps,
                                               const CoolDev* __restrict__ cool,
                                               const int64_t* __restrict__ counter,
                                               const int32_t* __restrict__ rb, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (rb && rb[i] >= 0) return;  // rigid-body members move with their body
    const TrapDev T = traps[0];
    const int64_t step = cool->step_base + *counter + 1;
    double4 p = src[i];
    double u = vx[i], v = vy[i], w = vz[i];
    half_step_drift(T, cool_switches<X>(cool), i, species[i], mass[i], step, p.x, p.y, p.z, u,
                    v, w, ax[i], ay[i],
                    az[i]);
    src[i] = p;
    vx[i] = u;
    vy[i] = v;
    vz[i] = w;
    if (srcm) srcm[i] = make_src(p.x, p.y, p.z, qe[i]);
}

// Inputs of the allocation-free force evaluation in the layout of the pair and
// epilogue kernels: the FP64 source stream {x, y, z, 1.5 q/e}, the FP32 stream
// (mixed precisions), Q/M and Q/e per ion (zero charge from n up to n_pad), and
// the trap parameters (written by thread 0).
__global__ __launch_bounds__(256) void k_pack_inputs(const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     const double* __restrict__ z,
                                                     const double* __restrict__ charge,
                                                     const double* __restrict__ mass, int64_t n,
                                                     int64_t n_pad, double4* __restrict__ src,
                                                     MixedSrc* __restrict__ srcm,
                                                     double* __restrict__ qm,
                                                     double* __restrict__ qe, TrapDev T,
                                                     TrapDev* __restrict__ tout) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *tout = T;
    if (i >= n_pad) return;
    if (i < n) {
        const double q = charge[i] / kElementaryCharge;
        src[i] = make_double4(x[i], y[i], z[i], 1.5 * q);
        if (srcm) srcm[i] = make_src(x[i], y[i], z[i], q);
        qm[i] = charge[i] / mass[i];
        qe[i] = q;
    } else {
        src[i] = make_double4(0.0, 0.0, 0.0, 0.0);
        if (srcm) srcm[i] = make_src(0.0, 0.0, 0.0, 0.0);
        qm[i] = 0.0;
        qe[i] = 0.0;
    }
}

__global__ __launch_bounds__(256) void k_pack_mixed(const double4* __restrict__ src,
                                                    MixedSrc* __restrict__ srcm,
                                                    const double* __restrict__ qe, int64_t n,
                                                    int64_t n_pad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    if (i < n) {
        const double4 p = src[i];
        srcm[i] = make_src(p.x, p.y, p.z, qe[i]);
    } else {
        srcm[i] = make_src(0.0, 0.0, 0.0, 0.0);
    }
}

// Pair-field kernels.  A block is 4 waves that share the same 64*I targets
// (lane l of every wave owns targets base + l + 64 k, k < I) and split the
// block's source slice [s*jps, s*jps + jps) four ways; the four partial sums
// are added in wave order through LDS and written once per slice.  Sources
// beyond N carry zero charge, so every range is a multiple of 64 sources.

constexpr int kWaves = 4;

// Sum the per-wave partials of 64*I targets in wave order; wave 0 stores.
// red must hold 3 * 3 * 64 * I doubles of LDS.
template <int I, typename PT = double>
__device__ __forceinline__ void reduce_store_in(double (&sx)[I], double (&sy)[I],
                                                double (&sz)[I], PT* __restrict__ part,
                                                int s, int64_t n, int64_t n_pad, int64_t base,
                                                double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave > 0) {
#pragma unroll
        for (int k = 0; k < I; ++k) {
            red[((wave - 1) * 3 + 0) * 64 * I + lane + 64 * k] = sx[k];
            red[((wave - 1) * 3 + 1) * 64 * I + lane + 64 * k] = sy[k];
            red[((wave - 1) * 3 + 2) * 64 * I + lane + 64 * k] = sz[k];
        }
    }
    __syncthreads();
    if (wave == 0) {
        PT* px = part + (int64_t)(3 * s) * n_pad;
#pragma unroll
        for (int k = 0; k < I; ++k) {
            double x = sx[k], y = sy[k], z = sz[k];
#pragma unroll
            for (int w = 0; w < kWaves - 1; ++w) {
                x += red[(w * 3 + 0) * 64 * I + lane + 64 * k];
                y += red[(w * 3 + 1) * 64 * I + lane + 64 * k];
                z += red[(w * 3 + 2) * 64 * I + lane + 64 * k];
            }
            const int64_t i = base + 64 * k;
            if (i < n) {
                px[i] = (PT)x;
                px[n_pad + i] = (PT)y;
                px[2 * n_pad + i] = (PT)z;
            }
        }
    }
}

template <int I, typename PT = double>
__device__ __forceinline__ void reduce_store(double (&sx)[I], double (&sy)[I], double (&sz)[I],
                                             PT* __restrict__ part, int s, int64_t n,
                                             int64_t n_pad, int64_t base) {
    __shared__ double red[(kWaves - 1) * 3 * 64 * I];
    reduce_store_in<I, PT>(sx, sy, sz, part, s, n, n_pad, base, red);
}

// Partials of the FP32 pair kernels: FP32 in the FP32 + FP64-run mode (each
// slice's or tile pair's FP64 sum rounded once when stored, the slices added in
// FP64 by the epilogue), FP64 in the compensated mode.
template <bool KAHAN>
__device__ __forceinline__ typename std::conditional<KAHAN, double, float>::type* mixed_partials(
    double* part) {
    return reinterpret_cast<typename std::conditional<KAHAN, double, float>::type*>(part);
}

// FP64: sources through scalar loads (wave-uniform addresses) into SGPRs; FP64
// VALU issues at the same rate with SGPR or VGPR operands.
template <int I>
__global__ __launch_bounds__(256) void k_pair_f64(const double4* __restrict__ src, int64_t n,
                                                  int n64, int jps, int64_t n_pad,
                                                  double* __restrict__ part,
                                                  int64_t* __restrict__ counter, BodyMask bm) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t base0 = (int64_t)blockIdx.x * (64 * I);
    const int64_t base = base0 + lane;
    const int s = blockIdx.y;
    const int part_len = jps / kWaves;
    const int jb = min(s * jps + wave * part_len, n64);
    const int je = min(jb + part_len, n64);
    double xi[I], yi[I], zi[I], sx[I], sy[I], sz[I];
    int ci[I];
#pragma unroll
    for (int k = 0; k < I; ++k) {
        const double4 p = src[base + 64 * k];
        xi[k] = p.x;
        yi[k] = p.y;
        zi[k] = p.z;
        sx[k] = sy[k] = sz[k] = 0.0;
        ci[k] = bm.code ? bm.code[base + 64 * k] : 0;
    }
    int tlo = 0, thi = -1;
    if (bm.code) target_body_range<I>(bm, base0, tlo, thi);
    for (int j16 = jb; j16 < je; j16 += 16) {
        if (!group_may_share_body(bm, j16 / 16, tlo, thi)) {
            for (int j = j16; j < j16 + 16; j += 4) {
                const double4 p0 = src[j], p1 = src[j + 1], p2 = src[j + 2], p3 = src[j + 3];
#pragma unroll
                for (int k = 0; k < I; ++k) {
                    pair_f64(p0, xi[k], yi[k], zi[k], sx[k], sy[k], sz[k]);
                    pair_f64(p1, xi[k], yi[k], zi[k], sx[k], sy[k], sz[k]);
                    pair_f64(p2, xi[k], yi[k], zi[k], sx[k], sy[k], sz[k]);
                    pair_f64(p3, xi[k], yi[k], zi[k], sx[k], sy[k], sz[k]);
                }
            }
        } else {
            for (int j = j16; j < j16 + 16; ++j) {
                const double4 p0 = src[j];
                const int cj = bm.code[j];
#pragma unroll
                for (int k = 0; k < I; ++k)
                    pair_f64_masked(p0, xi[k], yi[k], zi[k], ci[k], cj, sx[k], sy[k], sz[k]);
            }
        }
    }
    reduce_store<I>(sx, sy, sz, part, s, n, n_pad, base);
    if (counter && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *counter += 1;
}

// Accumulators of the FP32 pair path for I targets.
template <int I, bool KAHAN>
struct MixedAcc {
    double sx[I], sy[I], sz[I];           // FP64 sums (run flushes)
    float kx[I], ky[I], kz[I];            // Kahan sums
    float cx[I], cy[I], cz[I];            // Kahan compensations

    __device__ __forceinline__ void init() {
#pragma unroll
        for (int k = 0; k < I; ++k) {
            sx[k] = sy[k] = sz[k] = 0.0;
            kx[k] = ky[k] = kz[k] = cx[k] = cy[k] = cz[k] = 0.0f;
        }
    }
    __device__ __forceinline__ void finish() {
        if (KAHAN) {
#pragma unroll
            for (int k = 0; k < I; ++k) {
                sx[k] = (double)kx[k] - (double)cx[k];
                sy[k] = (double)ky[k] - (double)cy[k];
                sz[k] = (double)kz[k] - (double)cz[k];
            }
        }
    }
};

// One run of L sources from `q` (LDS or global) against I float-float targets.
// With MASK, cq[u] is the body code of source u and ci[k] that of target k;
// terms of ions sharing a body are dropped.
template <int I, int L, bool KAHAN, bool MASK = false, typename Src>
__device__ __forceinline__ void mixed_run(const Src* __restrict__ q, const FF (&t)[I],
                                          MixedAcc<I, KAHAN>& A,
                                          const int32_t* __restrict__ cq = nullptr,
                                          const int* ci = nullptr) {
    if (KAHAN) {
#pragma unroll
        for (int u = 0; u < L; ++u) {
            const MixedSrc m = q[u];
            const int cj = MASK ? cq[u] : 0;
#pragma unroll
            for (int k = 0; k < I; ++k) {
                float tx, ty, tz;
                pair_f32_terms(m, t[k], tx, ty, tz);
                if (MASK && ci[k] == cj) tx = ty = tz = 0.0f;
                kahan_add(tx, A.kx[k], A.cx[k]);
                kahan_add(ty, A.ky[k], A.cy[k]);
                kahan_add(tz, A.kz[k], A.cz[k]);
            }
        }
    } else {
        float fx[I], fy[I], fz[I];
#pragma unroll
        for (int k = 0; k < I; ++k) fx[k] = fy[k] = fz[k] = 0.0f;
#pragma unroll
        for (int u = 0; u < L; ++u) {
            const MixedSrc m = q[u];
            if (MASK) {
                const int cj = cq[u];
#pragma unroll
                for (int k = 0; k < I; ++k) {
                    float tx, ty, tz;
                    pair_f32_terms(m, t[k], tx, ty, tz);
                    if (ci[k] != cj) {
                        fx[k] += tx;
                        fy[k] += ty;
                        fz[k] += tz;
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < I; ++k) pair_f32(m, t[k], fx[k], fy[k], fz[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < I; ++k) {
            A.sx[k] += (double)fx[k];
            A.sy[k] += (double)fy[k];
            A.sz[k] += (double)fz[k];
        }
    }
}

template <int I>
__device__ __forceinline__ void load_targets(const MixedSrc* __restrict__ srcm, int64_t base,
                                             FF (&t)[I]) {
#pragma unroll
    for (int k = 0; k < I; ++k) {
        const MixedSrc m = srcm[base + 64 * k];
        t[k].xh = m.xh;
        t[k].yh = m.yh;
        t[k].zh = m.zh;
        t[k].xl = m.xl;
        t[k].yl = m.yl;
        t[k].zl = m.zl;
    }
}

// FP32 pair field, sources through scalar loads into SGPRs.  Every op that
// reads an SGPR issues at the single rate, so this variant is the reference
// for the LDS variant below.
template <int I, int L, bool KAHAN>
__global__ __launch_bounds__(256) void k_pair_mixed_s(const MixedSrc* __restrict__ srcm,
                                                      int64_t n, int n64, int jps,
                                                      int64_t n_pad, double* __restrict__ part,
                                                      int64_t* __restrict__ counter,
                                                      BodyMask bm) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t base0 = (int64_t)blockIdx.x * (64 * I);
    const int64_t base = base0 + lane;
    const int s = blockIdx.y;
    const int part_len = jps / kWaves;
    const int jb = min(s * jps + wave * part_len, n64);
    const int je = min(jb + part_len, n64);
    FF t[I];
    load_targets<I>(srcm, base, t);
    int ci[I];
#pragma unroll
    for (int k = 0; k < I; ++k) ci[k] = bm.code ? bm.code[base + 64 * k] : 0;
    int tlo = 0, thi = -1;
    if (bm.code) target_body_range<I>(bm, base0, tlo, thi);
    MixedAcc<I, KAHAN> A;
    A.init();
    for (int j16 = jb; j16 < je; j16 += 16) {
        if (!group_may_share_body(bm, j16 / 16, tlo, thi)) {
            for (int j = j16; j < j16 + 16; j += L) mixed_run<I, L, KAHAN>(srcm + j, t, A);
        } else {
            mixed_run<I, 16, KAHAN, true>(srcm + j16, t, A, bm.code + j16, ci);
        }
    }
    A.finish();
    reduce_store<I>(A.sx, A.sy, A.sz, mixed_partials<KAHAN>(part), s, n, n_pad, base);
    if (counter && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *counter += 1;
}

// FP32 pair field, sources staged in LDS tiles of kTile and read back with
// wave-uniform addresses (broadcast) into VGPRs, so that every FP32 op of the
// pair term has VGPR operands only and can dual-issue.
constexpr int kTile = 256;

template <int I, int L, bool KAHAN>
__global__ __launch_bounds__(256) void k_pair_mixed_l(const MixedSrc* __restrict__ srcm,
                                                      int64_t n, int n64, int jps,
                                                      int64_t n_pad, double* __restrict__ part,
                                                      int64_t* __restrict__ counter,
                                                      BodyMask bm) {
    __shared__ float4 tile[2 * kTile];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t base0 = (int64_t)blockIdx.x * (64 * I);
    const int64_t base = base0 + lane;
    const int s = blockIdx.y;
    const int jb = min(s * jps, n64);
    const int je = min(jb + jps, n64);
    FF t[I];
    load_targets<I>(srcm, base, t);
    int ci[I];
#pragma unroll
    for (int k = 0; k < I; ++k) ci[k] = bm.code ? bm.code[base + 64 * k] : 0;
    int tlo = 0, thi = -1;
    if (bm.code) target_body_range<I>(bm, base0, tlo, thi);
    MixedAcc<I, KAHAN> A;
    A.init();
    const float4* __restrict__ g = reinterpret_cast<const float4*>(srcm);
    const MixedSrc* tl = reinterpret_cast<const MixedSrc*>(tile);
    for (int j0 = jb; j0 < je; j0 += kTile) {
        const int cnt = min(kTile, je - j0);  // multiple of 64
        __syncthreads();
        for (int q = threadIdx.x; q < 2 * cnt; q += 256) tile[q] = g[2 * (int64_t)j0 + q];
        __syncthreads();
        const int per = cnt / kWaves;  // multiple of 16
        const MixedSrc* mine = tl + wave * per;
        const int g0 = j0 + wave * per;  // global index of the wave's first source
        for (int u16 = 0; u16 < per; u16 += 16) {
            if (!group_may_share_body(bm, (g0 + u16) / 16, tlo, thi)) {
                for (int u = u16; u < u16 + 16; u += L) mixed_run<I, L, KAHAN>(mine + u, t, A);
            } else {
                mixed_run<I, 16, KAHAN, true>(mine + u16, t, A, bm.code + g0 + u16, ci);
            }
        }
    }
    A.finish();
    reduce_store<I>(A.sx, A.sy, A.sz, mixed_partials<KAHAN>(part), s, n, n_pad, base);
    if (counter && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *counter += 1;
}

// ------------------------------------------------------------------
// Pair field with Newton's third law: every unordered pair is evaluated once.
//
// Ions are cut into tiles of 256.  Block u handles the tile pair (a, b), a <= b
// (the strict upper triangle row-major, then the diagonal tiles).  Its 4 waves
// each hold all 256 targets of tile a (4 per lane) and take 64 of the 256
// sources of tile b.  For a source j and
// target i the block adds q_j (r_i - r_j)/r^3 to target i (registers) and
// q_i (r_j - r_i)/r^3 to source j; the latter is summed over the wave's 64
// lanes through a per-wave LDS transpose (fixed order).  Diagonal tiles
// (a == b) evaluate all ordered pairs on the target side only.  Partial sums
// land in slot b for tile-a ions and in slot a for tile-b ions, so every ion
// receives exactly one partial per tile and the epilogue adds the nb slots in
// order: deterministic, no atomics.

constexpr int kSymTile = 256;

// Row a of off-diagonal unit u: rows r < a hold S(a) = a (nb - 1) - a (a - 1) / 2
// units, so a is the largest root bound of S(a) <= u, from the quadratic and
// then corrected by whole steps (in FP32 the estimate is already exact for
// nb <= 512, checked on the host for every unit).
__device__ __forceinline__ void sym_unit(int nb, int& a, int& b) {
    const int off = nb * (nb - 1) / 2;
    const int u = blockIdx.x;
    if (u >= off) {  // diagonal tiles, which skip the reaction sums, go last
        a = b = u - off;
        return;
    }
    auto rows_before = [nb](int r) { return r * (nb - 1) - r * (r - 1) / 2; };
    const float c = (float)nb - 0.5f;
    int r = (int)(c - sqrtf(fmaxf(c * c - 2.0f * (float)u, 0.0f)));
    r = min(max(r, 0), nb - 2);
    while (r + 1 <= nb - 2 && rows_before(r + 1) <= u) ++r;
    while (r > 0 && rows_before(r) > u) --r;
    a = r;
    b = r + 1 + (u - rows_before(r));
}

// Rigid-body exclusion for the pair-once kernels.  tile_body[t] is the body of
// every ion of tile t (>= 0) or -1 when the tile holds no body ions (bodies
// that share a tile with other ions take the all-pairs kernels instead).  A
// tile pair inside one body contributes nothing: its two partial slots get
// zeros, so the epilogue still adds one partial per tile.
__device__ __forceinline__ bool sym_unit_excluded(const int32_t* __restrict__ tile_body, int a,
                                                  int b) {
    return tile_body && tile_body[a] >= 0 && tile_body[a] == tile_body[b];
}

template <typename PT>
__device__ __forceinline__ void sym_unit_zero(PT* __restrict__ part, int64_t n, int64_t n_pad,
                                              int a, int b) {
    const int64_t i = (int64_t)a * kSymTile + threadIdx.x;  // target side, slot b
    if (i < n) {
        part[((int64_t)b * 3 + 0) * n_pad + i] = PT(0);
        part[((int64_t)b * 3 + 1) * n_pad + i] = PT(0);
        part[((int64_t)b * 3 + 2) * n_pad + i] = PT(0);
    }
    if (a != b) {  // reaction side, slot a
        const int64_t j = (int64_t)b * kSymTile + threadIdx.x;
        part[((int64_t)a * 3 + 0) * n_pad + j] = PT(0);
        part[((int64_t)a * 3 + 1) * n_pad + j] = PT(0);
        part[((int64_t)a * 3 + 2) * n_pad + j] = PT(0);
    }
}

// Body ids per tile for the masked pair-once path: tile pairs whose body-id
// ranges meet take the per-pair test, the others the plain loop.
struct BodyTiles {
    const int32_t* __restrict__ code = nullptr;  // [n_pad] body id, or -1 - i for free ion i
    const int32_t* __restrict__ tmin = nullptr;  // [tiles] smallest body id >= 0 in the tile
    const int32_t* __restrict__ tmax = nullptr;  // [tiles] largest (tmin > tmax: none)
    __device__ bool may_share(int a, int b) const {
        return tmin[a] <= tmax[b] && tmin[b] <= tmax[a];
    }
};

// Sum over the 64 lanes of a wave of C columns held lane-major in buf[64][S]
// (S = C + 1: consecutive lanes write consecutive rows, and a column read by
// consecutive lanes touches consecutive banks).  P lanes per column each add
// 64/P rows, then the P part sums are combined by lane exchanges (P = 2 or 4).
// FP64 rows are added in FP64 with four independent partial sums.  FP32 rows
// are added in FP32 runs of 8 (pairwise, so each run carries at most 3
// roundings) and the run totals in FP64, the same FP32-run / FP64-flush rule
// as the target sums.  The column total ends up in lanes with
// (lane % P) == 0, column = lane / P.
template <int C, int P, typename T, bool KH = false>
__device__ __forceinline__ double column_sum64(const T* __restrict__ buf, int lane) {
    static_assert(C * P <= 64 && (P == 2 || P == 4), "bad column split");
    constexpr int E = 64 / P, S = C + 1;
    const int col = lane / P, q = lane % P;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    if (col < C) {
        const T* p = buf + (E * q) * S + col;
        if constexpr (sizeof(T) == sizeof(float)) {
            static_assert(E % 8 == 0 && E / 8 <= 4, "FP32 runs of 8 rows");
            double run[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int g = 0; g < E / 8; ++g) {
                const T* r = p + 8 * g * S;
                const float s01 = r[0] + r[S], s23 = r[2 * S] + r[3 * S];
                const float s45 = r[4 * S] + r[5 * S], s67 = r[6 * S] + r[7 * S];
                run[g] = (double)((s01 + s23) + (s45 + s67));
            }
            if constexpr (KH) {
                // compensated FP32 sum of the run totals (the compensated mode)
                float ks = 0.0f, kc = 0.0f;
#pragma unroll
                for (int g = 0; g < E / 8; ++g) kahan_add((float)run[g], ks, kc);
                acc0 = (double)ks - (double)kc;
            } else {
                acc0 = run[0];
                acc1 = run[1];
                acc2 = run[2];
                acc3 = run[3];
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; e += 4) {
                acc0 += (double)p[(e + 0) * S];
                acc1 += (double)p[(e + 1) * S];
                acc2 += (double)p[(e + 2) * S];
                acc3 += (double)p[(e + 3) * S];
            }
        }
    }
    double acc = (acc0 + acc1) + (acc2 + acc3);
    acc += __shfl_xor(acc, 1);
    if (P == 4) acc += __shfl_xor(acc, 2);
    return acc;
}

// Target-side sums of the 4 targets per lane, added over the 4 waves in wave
// order through LDS in two halves (targets 0-1, then 2-3) and stored to the
// partial slot s.  red holds at least (kWaves - 1) * 3 * 64 * 2 doubles.
template <typename PT>
__device__ __forceinline__ void reduce_store_halves(double (&sx)[4], double (&sy)[4],
                                                    double (&sz)[4], PT* __restrict__ part,
                                                    int s, int64_t n, int64_t n_pad,
                                                    int64_t base, double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    PT* px = part + (int64_t)(3 * s) * n_pad;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (wave > 0) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                red[((wave - 1) * 3 + 0) * 128 + lane + 64 * k] = sx[2 * h + k];
                red[((wave - 1) * 3 + 1) * 128 + lane + 64 * k] = sy[2 * h + k];
                red[((wave - 1) * 3 + 2) * 128 + lane + 64 * k] = sz[2 * h + k];
            }
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                double x = sx[2 * h + k], y = sy[2 * h + k], z = sz[2 * h + k];
#pragma unroll
                for (int w = 0; w < kWaves - 1; ++w) {
                    x += red[(w * 3 + 0) * 128 + lane + 64 * k];
                    y += red[(w * 3 + 1) * 128 + lane + 64 * k];
                    z += red[(w * 3 + 2) * 128 + lane + 64 * k];
                }
                const int64_t i = base + 64 * (2 * h + k);
                if (i < n) {
                    px[i] = (PT)x;
                    px[n_pad + i] = (PT)y;
                    px[2 * n_pad + i] = (PT)z;
                }
            }
        }
        __syncthreads();
    }
}

// L: sources per FP32 run of the target sums (a multiple of CH), after which
// they go into the FP64 sums; CH: sources per reaction-sum chunk (LDS per block
// grows with it); WPE: the occupancy the register allocation aims at.
// FQ: every ion of the tile pair carries the same charge uq (in units of e), so
// the per-pair charge factors are applied once per sum instead (an exact
// refactoring; tiles holding zero-charge padding ions take the general path).
// MK: some pairs of the tile pair belong to one rigid body; code[i] is ion i's
// body id (or a number unique to a free ion) and a pair of equal codes adds 0.
// KH: the compensated mode, in which the FP32 runs are added in compensated
// FP32 (Kahan) instead of FP64 within the tile pair.
template <int L, int CH, int UNR, bool PF, bool FQ, bool MK = false, bool KH = false,
          typename PT = double>
__device__ __forceinline__ void mixed_sym_body(const MixedSrc* __restrict__ srcm, int64_t n,
                                               int nb, int64_t n_pad, PT* __restrict__ part,
                                               int a, int b, float uq, float4* tile,
                                               double* smem,
                                               const int32_t* __restrict__ code = nullptr,
                                               int32_t* tcode = nullptr) {
    constexpr int S = CH * 3 + 1;  // row stride of the lane-major reaction buffer
    const bool diag = (a == b);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)a * kSymTile + lane;
    FF t[4];
    float qi[4];
    int32_t ci[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const MixedSrc m = srcm[base + 64 * k];
        t[k].xh = m.xh;
        t[k].yh = m.yh;
        t[k].zh = m.zh;
        t[k].xl = m.xl;
        t[k].yl = m.yl;
        t[k].zl = m.zl;
        qi[k] = -m.nq;
        ci[k] = MK ? code[base + 64 * k] : 0;
    }
    {
        const float4* __restrict__ g = reinterpret_cast<const float4*>(srcm) + 2 * (int64_t)b * kSymTile;
        for (int q = threadIdx.x; q < 2 * kSymTile; q += 256) tile[q] = g[q];
        if constexpr (MK) tcode[threadIdx.x] = code[(int64_t)b * kSymTile + threadIdx.x];
    }
    __syncthreads();
    const MixedSrc* mine = reinterpret_cast<const MixedSrc*>(tile) + wave * 64;
    const int32_t* mcode = MK ? tcode + wave * 64 : nullptr;
    double sx[4], sy[4], sz[4];
    float ksx[4], ksy[4], ksz[4], kcx[4], kcy[4], kcz[4];  // KH: compensated target sums
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        sx[k] = sy[k] = sz[k] = 0.0;
        ksx[k] = ksy[k] = ksz[k] = kcx[k] = kcy[k] = kcz[k] = 0.0f;
    }
    float* jb = reinterpret_cast<float*>(smem) + wave * 64 * S;
    // with PF the next source is read from LDS while the current one is used
    MixedSrc m_next = mine[0];
    // target sums: FP32 runs of L sources (a multiple of CH), then into FP64
    static_assert(L % CH == 0 && 64 % L == 0, "runs of whole chunks");
    float fx[4], fy[4], fz[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) fx[k] = fy[k] = fz[k] = 0.0f;
    for (int s0 = 0; s0 < 64; s0 += CH) {
        if (KH) {
#pragma unroll
            for (int k = 0; k < 4; ++k) fx[k] = fy[k] = fz[k] = 0.0f;
        }
#pragma unroll UNR
        for (int uu = 0; uu < CH; ++uu) {
            MixedSrc m;
            if constexpr (PF) {
                m = m_next;
                m_next = mine[min(s0 + uu + 1, 63)];
            } else {
                m = mine[s0 + uu];
            }
            float tx = 0.0f, ty = 0.0f, tz = 0.0f;
            const int32_t cj = MK ? mcode[s0 + uu] : 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float dx = (m.xh - t[k].xh) + (m.xl - t[k].xl);
                const float dy = (m.yh - t[k].yh) + (m.yl - t[k].yl);
                const float dz = (m.zh - t[k].zh) + (m.zl - t[k].zl);
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, m.r2floor)));
                const float y = __builtin_amdgcn_rsqf(r2);
                const float y3 = (MK && ci[k] == cj) ? 0.0f : (y * y) * y;
                const float wi = FQ ? y3 : m.nq * y3;  // -q_j r^-3 (times -1/uq with FQ)
                fx[k] = fmaf(wi, dx, fx[k]);
                fy[k] = fmaf(wi, dy, fy[k]);
                fz[k] = fmaf(wi, dz, fz[k]);
                if (!diag) {
                    const float wj = FQ ? y3 : qi[k] * y3;  // q_i r^-3 (times 1/uq with FQ)
                    tx = fmaf(wj, dx, tx);
                    ty = fmaf(wj, dy, ty);
                    tz = fmaf(wj, dz, tz);
                }
            }
            if (!diag) {
                jb[lane * S + 3 * uu + 0] = tx;
                jb[lane * S + 3 * uu + 1] = ty;
                jb[lane * S + 3 * uu + 2] = tz;
            }
        }
        if constexpr (KH) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                kahan_add(fx[k], ksx[k], kcx[k]);
                kahan_add(fy[k], ksy[k], kcy[k]);
                kahan_add(fz[k], ksz[k], kcz[k]);
            }
        } else if ((s0 + CH) % L == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sx[k] += (double)fx[k];
                sy[k] += (double)fy[k];
                sz[k] += (double)fz[k];
                fx[k] = fy[k] = fz[k] = 0.0f;
            }
        }
        if (!diag) {
            // the wave's LDS writes are visible to all its lanes after this
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const double tot =
                column_sum64<CH * 3, (CH * 3 * 4 <= 64 ? 4 : 2), float, KH>(jb, lane);
            constexpr int P = CH * 3 * 4 <= 64 ? 4 : 2;
            const int col = lane / P;
            if ((lane % P) == 0 && col < CH * 3) {
                const int uu = col / 3, c = col - 3 * uu;
                const int64_t j = (int64_t)b * kSymTile + wave * 64 + s0 + uu;
                part[((int64_t)a * 3 + c) * n_pad + j] = (PT)(FQ ? tot * (double)uq : tot);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    if constexpr (KH) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sx[k] = (double)ksx[k] - (double)kcx[k];
            sy[k] = (double)ksy[k] - (double)kcy[k];
            sz[k] = (double)ksz[k] - (double)kcz[k];
        }
    }
    if (FQ) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sx[k] *= -(double)uq;
            sy[k] *= -(double)uq;
            sz[k] *= -(double)uq;
        }
    }
    __syncthreads();  // every wave is done with its reaction buffer
    reduce_store_halves(sx, sy, sz, part, b, n, n_pad, base, smem);
}

// uq != 0: every ion carries the charge uq (units of e) and tiles below
// full_tiles hold no padding; those tile pairs take the charge-free loop.
template <int L, int CH, int WPE, int UNR, bool PF = false, bool MK = false, bool KH = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_pair_mixed_sym(const MixedSrc* __restrict__ srcm, int64_t n, int nb, int64_t n_pad,
                      double* __restrict__ part, int64_t* __restrict__ counter, float uq,
                      int full_tiles, const int32_t* __restrict__ tile_body,
                      const BodyTiles bt = BodyTiles{}) {
    __shared__ int32_t tcode[MK ? kSymTile : 1];
    __shared__ float4 tile[2 * kSymTile];
    // per-wave reaction buffers, reused for the final target-side reduction
    constexpr int S = CH * 3 + 1;
    constexpr int kRed = (kWaves - 1) * 3 * 64 * 2;
    constexpr int kBuf = (kWaves * 64 * S + 1) / 2;
    __shared__ __align__(16) double smem[kBuf > kRed ? kBuf : kRed];
    auto* pt = mixed_partials<KH>(part);
    int a, b;
    sym_unit(nb, a, b);
    if (sym_unit_excluded(tile_body, a, b))
        sym_unit_zero(pt, n, n_pad, a, b);
    else if (MK && bt.may_share(a, b))
        mixed_sym_body<L, CH, UNR, PF, false, true, KH>(srcm, n, nb, n_pad, pt, a, b, uq, tile,
                                                        smem, bt.code, tcode);
    else if (uq != 0.0f && b < full_tiles)
        mixed_sym_body<L, CH, UNR, PF, true, false, KH>(srcm, n, nb, n_pad, pt, a, b, uq, tile,
                                                        smem);
    else
        mixed_sym_body<L, CH, UNR, PF, false, false, KH>(srcm, n, nb, n_pad, pt, a, b, uq, tile,
                                                         smem);
    if (counter && blockIdx.x == 0 && threadIdx.x == 0) *counter += 1;
}

// One tile pair (a, b) of the FP64 pair-once kernel.  With FQ every ion in
// both tiles carries the charge uq: the sums run over c d alone and are scaled
// by the charge once, at the end.
template <int UNR, bool PF, bool FQ, bool MK, bool DG>
__device__ __forceinline__ void f64_sym_body(const double4* __restrict__ src,
                                             const double* __restrict__ qe, int64_t n,
                                             int64_t n_pad, double* __restrict__ part, int a,
                                             int b, double uq, double* smem,
                                             const int32_t* __restrict__ code = nullptr) {
    constexpr int CH = 4;
    constexpr int S = CH * 3 + 1;
    constexpr bool diag = DG;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t base = (int64_t)a * kSymTile + lane;
    double xi[4], yi[4], zi[4], nqi[4], sx[4], sy[4], sz[4];
    int32_t ci[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double4 p = src[base + 64 * k];
        xi[k] = p.x;
        yi[k] = p.y;
        zi[k] = p.z;
        nqi[k] = FQ ? 0.0 : -1.5 * qe[base + 64 * k];
        ci[k] = MK ? code[base + 64 * k] : 0;
        sx[k] = sy[k] = sz[k] = 0.0;
    }
    double* jb = smem + wave * 64 * S;
    const int64_t j0 = (int64_t)b * kSymTile + wave * 64;
    // with PF the next source is loaded while the current one is used
    double4 p_next = src[j0];
    for (int s0 = 0; s0 < 64; s0 += CH) {
#pragma unroll UNR
        for (int uu = 0; uu < CH; ++uu) {
            double4 p;
            if constexpr (PF) {
                p = p_next;
                p_next = src[j0 + min(s0 + uu + 1, 63)];
            } else {
                p = src[j0 + s0 + uu];
            }
            double tx = 0.0, ty = 0.0, tz = 0.0;
            const int32_t cj = MK ? code[j0 + s0 + uu] : 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double dx = p.x - xi[k], dy = p.y - yi[k], dz = p.z - zi[k];
                const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, kR2FloorF64)));
                const double y = __builtin_amdgcn_rsq(r2);
                const double a2 = y * y;
                const double g = fma(r2, a2, -5.0 / 3.0);
                // -(2/3) r^-3 (one Newton correction); 0 for a pair inside one body
                const double c = (MK && ci[k] == cj) ? 0.0 : (a2 * y) * g;
                const double wi = FQ ? c : c * p.w;  // 1.5 q_j c = -q_j r^-3
                sx[k] = fma(wi, dx, sx[k]);
                sy[k] = fma(wi, dy, sy[k]);
                sz[k] = fma(wi, dz, sz[k]);
                if constexpr (!diag) {
                    const double wj = FQ ? c : c * nqi[k];  // -1.5 q_i c = q_i r^-3
                    tx = fma(wj, dx, tx);
                    ty = fma(wj, dy, ty);
                    tz = fma(wj, dz, tz);
                }
            }
            if constexpr (!diag) {
                jb[lane * S + 3 * uu + 0] = tx;
                jb[lane * S + 3 * uu + 1] = ty;
                jb[lane * S + 3 * uu + 2] = tz;
            }
        }
        if constexpr (!diag) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const double tot = column_sum64<CH * 3, 4>(jb, lane);
            const int col = lane >> 2;
            if ((lane & 3) == 0 && col < CH * 3) {
                const int uu = col / 3, c = col - 3 * uu;
                part[((int64_t)a * 3 + c) * n_pad + j0 + s0 + uu] = FQ ? tot * (-1.5 * uq) : tot;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    if (FQ) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sx[k] *= 1.5 * uq;
            sy[k] *= 1.5 * uq;
            sz[k] *= 1.5 * uq;
        }
    }
    __syncthreads();  // every wave is done with its reaction buffer
    reduce_store_in<4>(sx, sy, sz, part, b, n, n_pad, base, smem);
}

// A diagonal tile pair (a == b) adds no reactions: it gets a loop of its own,
// so the loop of the other tile pairs carries no branch on it.
template <int UNR, bool PF, bool FQ, bool MK>
__device__ __forceinline__ void f64_sym_unit(const double4* __restrict__ src,
                                             const double* __restrict__ qe, int64_t n,
                                             int64_t n_pad, double* __restrict__ part, int a,
                                             int b, double uq, double* smem,
                                             const int32_t* __restrict__ code = nullptr) {
    if (a == b)
        f64_sym_body<UNR, PF, FQ, MK, true>(src, qe, n, n_pad, part, a, b, uq, smem, code);
    else
        f64_sym_body<UNR, PF, FQ, MK, false>(src, qe, n, n_pad, part, a, b, uq, smem, code);
}

// WPE: the occupancy the register allocation aims at; UNR: sources unrolled.
// uq != 0: every ion carries the charge uq (units of e) and tiles below
// full_tiles hold no padding; those tile pairs take the charge-free loop.
template <int WPE, int UNR, bool PF = false, bool MK = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_pair_f64_sym(const double4* __restrict__ src, const double* __restrict__ qe, int64_t n,
                    int nb, int64_t n_pad, double* __restrict__ part,
                    int64_t* __restrict__ counter, double uq, int full_tiles,
                    const int32_t* __restrict__ tile_body, const BodyTiles bt = BodyTiles{}) {
    constexpr int S = 4 * 3 + 1;
    __shared__ double smem[kWaves * 64 * S];
    static_assert(kWaves * 64 * S >= (kWaves - 1) * 3 * 64 * 4, "LDS reuse too small");
    int a, b;
    sym_unit(nb, a, b);
    if (sym_unit_excluded(tile_body, a, b))
        sym_unit_zero(part, n, n_pad, a, b);
    else if (MK && bt.may_share(a, b))
        f64_sym_unit<UNR, PF, false, true>(src, qe, n, n_pad, part, a, b, uq, smem, bt.code);
    else if (uq != 0.0 && b < full_tiles)
        f64_sym_unit<UNR, PF, true, false>(src, qe, n, n_pad, part, a, b, uq, smem);
    else
        f64_sym_unit<UNR, PF, false, false>(src, qe, n, n_pad, part, a, b, uq, smem);
    if (counter && blockIdx.x == 0 && threadIdx.x == 0) *counter += 1;
}

// The per-ion inputs of the end of a step.
struct IonIn {
    double4 p;  // position (w: the FP64 source weight, carried along)
    double u, v, w, qm, qe, mass;
    int32_t sp;
};

__device__ __forceinline__ IonIn load_ion(int64_t i, const double4* src_in,
                                          const double* __restrict__ vx,
                                          const double* __restrict__ vy,
                                          const double* __restrict__ vz,
                                          const double* __restrict__ qm,
                                          const double* __restrict__ qe,
                                          const double* __restrict__ mass,
                                          const int32_t* __restrict__ species) {
    IonIn r;
    r.p = src_in[i];
    r.u = vx[i];
    r.v = vy[i];
    r.w = vz[i];
    r.qm = qm[i];
    r.qe = qe[i];
    r.mass = mass[i];
    r.sp = species[i];
    return r;
}

// The end of a step for ion i (inputs in) from its summed pair field S
// (scaled), with c = cos(Omega t) of the step's time: the trap field, then
// (mode kModeEnd) the closing half kick with damping, or (kModeEndDrift) also
// the first half of the next step, whose position goes to src_out;
// kModeAccel stores the acceleration only.  kc is the call's step counter
// after this step (numbers the cooling draws).
template <bool X>
__device__ __forceinline__ void end_step_vals(
    int mode, int64_t i, int64_t kc, const TrapDev& T, double c, double Sx, double Sy,
    double Sz, IonIn in, double4* src_out, MixedSrc* __restrict__ srcm_out,
    double* __restrict__ vx, double* __restrict__ vy, double* __restrict__ vz,
    double* __restrict__ ax, double* __restrict__ ay, double* __restrict__ az, int64_t n_pad,
    const CoolDev* __restrict__ cool, double* __restrict__ vacc, double* __restrict__ vavg) {
    double4 p = in.p;
    double a_x, a_y, a_z;
    trap_accel_c(T, c, in.qm, p.x, p.y, p.z, Sx, Sy, Sz, a_x, a_y, a_z);
    ax[i] = a_x;
    ay[i] = a_y;
    az[i] = a_z;
    if (mode == kModeAccel) return;
    const int64_t step = cool->step_base + kc;  // the step this epilogue completes
    double u = in.u, v = in.v, w = in.w;
    const CoolRef cr = cool_switches<X>(cool);
    end_kick(T, cr, i, in.sp, in.mass, step, u, v, w, a_x, a_y, a_z);
    time_average(cr, i, n_pad, step, vacc, vavg, u, v, w);
    if (mode == kModeEndDrift) {
        half_step_drift(T, cr, i, in.sp, in.mass, step + 1, p.x, p.y, p.z, u, v, w, a_x, a_y,
                        a_z);
        src_out[i] = p;
        if (srcm_out) srcm_out[i] = make_src(p.x, p.y, p.z, in.qe);
    }
    vx[i] = u;
    vy[i] = v;
    vz[i] = w;
}

// As end_step_vals, loading the inputs first; rigid-body members (rb[i] >= 0)
// only get their acceleration (their body kicks them).
template <bool X>
__device__ __forceinline__ void end_step_ion(
    int mode, int64_t i, int64_t kc, const TrapDev& T, double t, double Sx, double Sy,
    double Sz, const double4* src_in, double4* src_out, MixedSrc* __restrict__ srcm_out,
    double* __restrict__ vx, double* __restrict__ vy, double* __restrict__ vz,
    double* __restrict__ ax, double* __restrict__ ay, double* __restrict__ az,
    const double* __restrict__ qm, const double* __restrict__ qe,
    const double* __restrict__ mass, const int32_t* __restrict__ species, int64_t n_pad,
    const CoolDev* __restrict__ cool, double* __restrict__ vacc, double* __restrict__ vavg,
    const int32_t* __restrict__ rb) {
    const IonIn in = load_ion(i, src_in, vx, vy, vz, qm, qe, mass, species);
    const double c = T.ps != 0.0 ? 0.0 : cos(T.omega * t);
    const int m = (mode != kModeAccel && rb && rb[i] >= 0) ? kModeAccel : mode;
    end_step_vals<X>(m, i, kc, T, c, Sx, Sy, Sz, in, src_out, srcm_out, vx, vy, vz, ax, ay, az,
                     n_pad, cool, vacc, vavg);
}

// Per-ion epilogue of a step (or a plain force evaluation): reduce the slice
// partials in slice order, add the trap field, then kick / damp / drift.
// Per-ion epilogue of a step (or a plain force evaluation).  A block covers 64
// ions with 4 waves: wave g adds the partial slots [g*per, (g+1)*per) in slot
// order, wave 0 adds the four group sums in group order (deterministic for a
// given number of slots), then applies the trap field and kick / damp / drift.
template <int MODE, int UW, bool X, typename PT = double>
__global__ __launch_bounds__(64 * UW) void k_update(double4* __restrict__ src,
                                                MixedSrc* __restrict__ srcm,
                                                double* __restrict__ vx, double* __restrict__ vy,
                                                double* __restrict__ vz, double* __restrict__ ax,
                                                double* __restrict__ ay, double* __restrict__ az,
                                                const double* __restrict__ qm,
                                                const double* __restrict__ qe,
                                                const double* __restrict__ mass,
                                                const int32_t* __restrict__ species,
                                                const PT* __restrict__ part, int j_split,
                                                int64_t n, int64_t n_pad, double field_scale,
                                                const TrapDev* __restrict__ traps,
                                                const CoolDev* __restrict__ cool,
                                                const int64_t* __restrict__ counter,
                                                double* __restrict__ vacc,
                                                double* __restrict__ vavg,
                                                const int32_t* __restrict__ rb) {
    // UW waves per 64 ions: wave g sums a contiguous range of slices, then the
    // wave sums are added in wave order
    __shared__ double red[UW - 1][3][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    const int per = (j_split + UW - 1) / UW;
    const int s0 = min(g * per, j_split), s1 = min(s0 + per, j_split);
    double Sx = 0.0, Sy = 0.0, Sz = 0.0;
    if (i < n) {
#pragma unroll 4
        for (int s = s0; s < s1; ++s) {
            const PT* px = part + (int64_t)(3 * s) * n_pad;
            Sx += (double)px[i];
            Sy += (double)px[n_pad + i];
            Sz += (double)px[2 * n_pad + i];
        }
    }
    if (g > 0) {
        red[g - 1][0][lane] = Sx;
        red[g - 1][1][lane] = Sy;
        red[g - 1][2][lane] = Sz;
    }
    __syncthreads();
    if (g > 0 || i >= n) return;
#pragma unroll
    for (int w = 0; w < UW - 1; ++w) {
        Sx += red[w][0][lane];
        Sy += red[w][1][lane];
        Sz += red[w][2][lane];
    }
    const TrapDev T = traps[0];
    const double t = counter ? T.t_start + (double)(*counter) * T.dt : T.t_start;
    end_step_ion<X>(MODE, i, counter ? *counter : 0, T, t, Sx * field_scale, Sy * field_scale,
                    Sz * field_scale, src, src, srcm, vx, vy, vz, ax, ay, az, qm, qe, mass,
                    species, n_pad, cool, vacc, vavg, rb);
}

// ---------------------------------------------- one launch per step (mid-size traps)
//
// One trap of n ions, one launch per step.  Workgroup g owns the TR targets
// [g TR, g TR + TR); thread t takes the sources t, t + kRowsBlock, ... for all
// of them.  The per-thread sums are added over each wave by a fixed butterfly
// (every lane ends with the same sum) and over the waves in wave order, and the
// owning threads end the step for their targets.  Every workgroup reads all
// positions of the step, so the drifted positions go to the other buffer.

constexpr int kRowsBlock = 256;

struct RowsArgs {
    const double4* src_in;
    double4* src_out;        // drifted positions (kModeEndDrift), or the home buffer
    const MixedSrc* srcm_in;
    MixedSrc* srcm_out;
    double *vx, *vy, *vz, *ax, *ay, *az;
    const double *qm, *qe, *mass;
    const int32_t* species;
    const TrapDev* traps;
    const CoolDev* cool;
    const int64_t* counter;  // the call's step counter at the start of the chunk
    double *vacc, *vavg;
    int64_t n, n_pad;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <int PREC, int TR, bool X>
__global__ __launch_bounds__(kRowsBlock) void k_rows(const RowsArgs A, int mode, int k_in_chunk) {
    __shared__ double red[kRowsBlock / 64][3 * TR];
    const int64_t n = A.n;
    const int64_t i0 = (int64_t)blockIdx.x * TR;
    const int tid = threadIdx.x;
    // the owners' inputs and the step's time first, so that their loads overlap
    // the pair work
    const TrapDev T = A.traps[0];
    const bool counted = mode != kModeAccel;
    const int64_t kc = counted ? *A.counter + k_in_chunk + 1 : 0;
    const bool own = tid < TR && i0 + tid < n;
    IonIn me{};
    if (own)
        me = load_ion(i0 + tid, A.src_in, A.vx, A.vy, A.vz, A.qm, A.qe, A.mass, A.species);
    double sx[TR], sy[TR], sz[TR];
#pragma unroll
    for (int k = 0; k < TR; ++k) sx[k] = sy[k] = sz[k] = 0.0;
    // sources four at a time (all four loads in flight); past n the last ion again,
    // with zero weight
    constexpr int U = 4;
    if constexpr (PREC == 0) {
        double tx[TR], ty[TR], tz[TR];
#pragma unroll
        for (int k = 0; k < TR; ++k) {
            const double4 p = A.src_in[min(i0 + k, n - 1)];
            tx[k] = p.x;
            ty[k] = p.y;
            tz[k] = p.z;
        }
        for (int64_t j0 = tid; j0 < n; j0 += U * kRowsBlock) {
            double4 P[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t j = j0 + (int64_t)u * kRowsBlock;
                P[u] = A.src_in[min(j, n - 1)];
                if (j >= n) P[u].w = 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < TR; ++k)
                    pair_f64(P[u], tx[k], ty[k], tz[k], sx[k], sy[k], sz[k]);
        }
    } else {
        FF tf[TR];
#pragma unroll
        for (int k = 0; k < TR; ++k) {
            const MixedSrc m = A.srcm_in[min(i0 + k, n - 1)];
            tf[k] = FF{m.xh, m.yh, m.zh, m.xl, m.yl, m.zl};
        }
        float fx[TR], fy[TR], fz[TR], cx[TR], cy[TR], cz[TR];
#pragma unroll
        for (int k = 0; k < TR; ++k) fx[k] = fy[k] = fz[k] = cx[k] = cy[k] = cz[k] = 0.0f;
        int run = 0;
        for (int64_t j0 = tid; j0 < n; j0 += U * kRowsBlock) {
            MixedSrc Q[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t j = j0 + (int64_t)u * kRowsBlock;
                Q[u] = A.srcm_in[min(j, n - 1)];
                if (j >= n) Q[u].nq = 0.0f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int k = 0; k < TR; ++k) {
                    if constexpr (PREC == 2) {
                        float ux, uy, uz;
                        pair_f32_terms(Q[u], tf[k], ux, uy, uz);
                        kahan_add(ux, fx[k], cx[k]);
                        kahan_add(uy, fy[k], cy[k]);
                        kahan_add(uz, fz[k], cz[k]);
                    } else {
                        pair_f32(Q[u], tf[k], fx[k], fy[k], fz[k]);
                    }
                }
            }
            // FP32 runs of 8 sources, flushed to FP64 (compensated: one run)
            run += U;
            if (PREC == 1 && run == 8) {
                run = 0;
#pragma unroll
                for (int k = 0; k < TR; ++k) {
                    sx[k] += (double)fx[k];
                    sy[k] += (double)fy[k];
                    sz[k] += (double)fz[k];
                    fx[k] = fy[k] = fz[k] = 0.0f;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < TR; ++k) {
            sx[k] += (double)fx[k] - (double)cx[k];
            sy[k] += (double)fy[k] - (double)cy[k];
            sz[k] += (double)fz[k] - (double)cz[k];
        }
    }
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int k = 0; k < TR; ++k) {
        const double x = wave_sum(sx[k]), y = wave_sum(sy[k]), z = wave_sum(sz[k]);
        if (lane == 0) {
            red[wave][3 * k + 0] = x;
            red[wave][3 * k + 1] = y;
            red[wave][3 * k + 2] = z;
        }
    }
    const double t = counted ? T.t_start + (double)kc * T.dt : T.t_start;
    const double crf = (own && T.ps == 0.0) ? cos(T.omega * t) : 0.0;
    __syncthreads();
    if (!own) return;
    const int k = tid;
    double Sx = red[0][3 * k], Sy = red[0][3 * k + 1], Sz = red[0][3 * k + 2];
#pragma unroll
    for (int w = 1; w < kRowsBlock / 64; ++w) {
        Sx += red[w][3 * k];
        Sy += red[w][3 * k + 1];
        Sz += red[w][3 * k + 2];
    }
    const double fs = PREC == 0 ? 1.0 : kMixedFieldScale;
    const int64_t i = i0 + k;
    end_step_vals<X>(mode, i, kc, T, crf, Sx * fs, Sy * fs, Sz * fs, me, A.src_out, A.srcm_out,
                     A.vx, A.vy, A.vz, A.ax, A.ay, A.az, A.n_pad, A.cool, A.vacc, A.vavg);
    // the last step of a launch sequence leaves the positions in the home buffer
    if (mode == kModeEnd && A.src_out != A.src_in) {
        A.src_out[i] = me.p;
        if (A.srcm_out) A.srcm_out[i] = A.srcm_in[i];
    }
}

__global__ void k_counter_add(int64_t* counter, int64_t k) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter += k;
}

// Coulomb potential sum_{j != i, same trap} q_j / r_ij per ion (1/m), FP64.
__global__ __launch_bounds__(256) void k_coulomb_potential(const double4* __restrict__ src,
                                                           const double* __restrict__ qe,
                                                           const int32_t* __restrict__ trap_of,
                                                           const int64_t* __restrict__ offsets,
                                                           int64_t n, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int tr = trap_of[i];
    const int64_t jb = offsets[tr], je = offsets[tr + 1];
    const double4 p = src[i];
    double acc = 0.0;
    for (int64_t j = jb; j < je; ++j) {
        if (j == i) continue;
        const double4 q = src[j];
        const double dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 == 0.0) continue;
        acc += qe[j] / sqrt(r2);
    }
    out[i] = acc;
}

__global__ __launch_bounds__(256) void k_check_finite(const double4* __restrict__ src,
                                                      const double* __restrict__ vx,
                                                      const double* __restrict__ vy,
                                                      const double* __restrict__ vz, int64_t n,
                                                      int32_t* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 p = src[i];
    const bool ok = isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(vx[i]) &&
                    isfinite(vy[i]) && isfinite(vz[i]);
    if (!ok) atomicAdd(flags, 1);
}

// Lost-ion check: ions farther than sqrt(r2_lost) from the trap centre, or
// with a non-finite position, are counted into *count.
__global__ __launch_bounds__(256) void k_count_lost(const double4* __restrict__ src, int64_t n,
                                                    double r2_lost, int32_t* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 p = src[i];
    const double r2 = p.x * p.x + p.y * p.y + p.z * p.z;
    if (!(r2 <= r2_lost)) atomicAdd(count, 1);
}

// ------------------------------------------------------------ batched traps
//
// One workgroup per trap, launched largest trap first so that the hardware
// dispatcher hands the long traps out before the short ones.  Threads form
// (i_slot, j_part) pairs: IS = min(round_up(m, 64), BLOCK) target slots and
// JP = BLOCK / IS source parts.  Slot owners (j_part 0) keep their ions' state
// in registers for the whole launch; the trap's source stream lives in LDS.

constexpr int kMaxTrap = 1024;
// Traps of at least kBatchTpt4 (kBatchTpt2) ions give each thread 4 (2) targets.
constexpr int kBatchTpt4 = 256;
constexpr int kBatchTpt2 = 128;


// One source of the batched FP32 pair loops: the position scaled by 2^20 per
// metre (exact) in FP64, so that the difference to a target is formed in FP64
// and rounded once to FP32 (three FP64 subtractions and three conversions per
// pair, against nine FP32 operations on float-float parts), then the negated
// charge and the r^2 floor as FP32 operands.
struct BatchMixedSrc {
    double x, y, z;
    float nq, r2floor;
};

// Whether the batched loops of precision prec factor a common charge out of
// the pair sums: FP64 and FP32 + FP64 runs (the 512-trap batch: 34.8 against
// 35.4 us and 29.8 against 30.2 us per step); not the compensated mode, whose
// loop measured 10 % slower without the charge multiply.
__device__ __forceinline__ bool batch_fq_on(int prec) { return prec != 2; }

template <int PREC>
struct BatchSrc;
template <>
struct BatchSrc<0> {
    using T = double4;
};
template <>
struct BatchSrc<1> {
    using T = BatchMixedSrc;
};
template <>
struct BatchSrc<2> {
    using T = MixedSrc;  // the compensated mode keeps float-float differences
};

__device__ __forceinline__ BatchMixedSrc make_batch_src(double x, double y, double z, double qe) {
    BatchMixedSrc s;
    s.x = x * kMixedScale;
    s.y = y * kMixedScale;
    s.z = z * kMixedScale;
    s.nq = (float)(-qe);
    s.r2floor = kR2FloorF32;
    return s;
}

// One FP32 pair term from a batched source: d rounded once from the FP64
// difference; returns r^-3 d (UNIT) or -q r^-3 d in (tx, ty, tz).
template <bool UNIT>
__device__ __forceinline__ void batch_pair_f32(const BatchMixedSrc& p, double xi, double yi,
                                               double zi, float& tx, float& ty, float& tz) {
    const float dx = (float)(p.x - xi), dy = (float)(p.y - yi), dz = (float)(p.z - zi);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, p.r2floor)));
    const float y = __builtin_amdgcn_rsqf(r2);
    const float w = UNIT ? y * (y * y) : (p.nq * y) * (y * y);
    tx = w * dx;
    ty = w * dy;
    tz = w * dz;
}

// FP32 sums of runs of RUN sources over [jb, je), each run added to the FP64
// sums (sx, sy, sz) of its target; the last run as far as the sources go.
// Within a run the sources go 8 at a time (unrolled), then one by one.
template <int TPT, bool FQ, int RUN>
__device__ __forceinline__ void batch_runs_f32(const BatchMixedSrc* __restrict__ lds, int jb,
                                               int je, const double (&xi)[TPT],
                                               const double (&yi)[TPT], const double (&zi)[TPT],
                                               double (&sx)[TPT], double (&sy)[TPT],
                                               double (&sz)[TPT]) {
    for (int j = jb; j < je; j += RUN) {
        float fx[TPT], fy[TPT], fz[TPT];
#pragma unroll
        for (int k = 0; k < TPT; ++k) fx[k] = fy[k] = fz[k] = 0.0f;
        const int jend = min(j + RUN, je);
        for (int j8 = j; j8 < jend; j8 += 8) {
            if (j8 + 8 <= jend) {
#pragma unroll
                for (int uu = 0; uu < 8; ++uu) {
                    const BatchMixedSrc q = lds[j8 + uu];
#pragma unroll
                    for (int k = 0; k < TPT; ++k) {
                        float tx, ty, tz;
                        batch_pair_f32<FQ>(q, xi[k], yi[k], zi[k], tx, ty, tz);
                        fx[k] += tx;
                        fy[k] += ty;
                        fz[k] += tz;
                    }
                }
            } else {
                for (int jj = j8; jj < jend; ++jj) {
                    const BatchMixedSrc q = lds[jj];
#pragma unroll
                    for (int k = 0; k < TPT; ++k) {
                        float tx, ty, tz;
                        batch_pair_f32<FQ>(q, xi[k], yi[k], zi[k], tx, ty, tz);
                        fx[k] += tx;
                        fy[k] += ty;
                        fz[k] += tz;
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            sx[k] += (double)fx[k];
            sy[k] += (double)fy[k];
            sz[k] += (double)fz[k];
        }
    }
}

// Field sums of TPT targets per thread over the sources [jb, je) of the LDS
// stream (je <= m: only the trap's ions, no padding): each source is read once
// for all TPT targets (il_k = slot + ws k),
// which cuts the broadcast LDS reads per pair by TPT.  Per target the sums run
// over the sources in order, as with one target per thread (FP32 runs
// flushed to FP64, or Kahan).  Targets at or beyond m give unused sums.
// FQ: every ion carries the charge uq (units of e); the sums run over r^-3 d
// alone and are scaled by the charge once.
template <int PREC, int TPT, bool FQ>
__device__ __forceinline__ void batch_pairs_multi(const typename BatchSrc<PREC>::T* __restrict__ lds,
                                                  int m, int slot, int ws, int jb, int je,
                                                  double uq, double (&Sx)[4], double (&Sy)[4],
                                                  double (&Sz)[4]) {
    int il[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int t = slot + ws * k;
        il[k] = t < m ? t : 0;
    }
    if constexpr (PREC == 0) {
        double xi[TPT], yi[TPT], zi[TPT], sx[TPT], sy[TPT], sz[TPT];
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            const double4 me = lds[il[k]];
            xi[k] = me.x;
            yi[k] = me.y;
            zi[k] = me.z;
            sx[k] = sy[k] = sz[k] = 0.0;
        }
        // sources four at a time, then the last one to three
        const int j4 = jb + ((je - jb) & ~3);
        for (int j = jb; j < j4; j += 4) {
#pragma unroll
            for (int uu = 0; uu < 4; ++uu) {
                const double4 p = lds[j + uu];
#pragma unroll
                for (int k = 0; k < TPT; ++k) {
                    if constexpr (FQ)
                        pair_f64_unit(p, xi[k], yi[k], zi[k], sx[k], sy[k], sz[k]);
                    else
                        pair_f64(p, xi[k], yi[k], zi[k], sx[k], sy[k], sz[k]);
                }
            }
        }
        for (int j = j4; j < je; ++j) {
            const double4 p = lds[j];
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                if constexpr (FQ)
                    pair_f64_unit(p, xi[k], yi[k], zi[k], sx[k], sy[k], sz[k]);
                else
                    pair_f64(p, xi[k], yi[k], zi[k], sx[k], sy[k], sz[k]);
            }
        }
        const double cq = FQ ? 1.5 * uq : 1.0;  // pair_f64_unit leaves out the 1.5 q_j factor
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            Sx[k] = FQ ? sx[k] * cq : sx[k];
            Sy[k] = FQ ? sy[k] * cq : sy[k];
            Sz[k] = FQ ? sz[k] * cq : sz[k];
        }
    } else {
        // the unit-weight terms leave out the -q_j factor
        const double cs = FQ ? -uq * kMixedFieldScale : kMixedFieldScale;
        if constexpr (PREC == 1) {
            double xi[TPT], yi[TPT], zi[TPT];
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                const BatchMixedSrc me = lds[il[k]];
                xi[k] = me.x;
                yi[k] = me.y;
                zi[k] = me.z;
            }
            double sx[TPT], sy[TPT], sz[TPT];
#pragma unroll
            for (int k = 0; k < TPT; ++k) sx[k] = sy[k] = sz[k] = 0.0;
            // FP32 runs flushed to FP64 (the last one shorter): 16 sources with
            // several targets per thread (large traps), else 8.  On the 512-trap
            // batch, M1 against the FP64 path 3.7e-7 with runs of 16, 5.0e-7 with
            // runs of 32 or 64, 3.3e-7 with runs of 8.
            if constexpr (TPT > 1)
                batch_runs_f32<TPT, FQ, 16>(lds, jb, je, xi, yi, zi, sx, sy, sz);
            else
                batch_runs_f32<TPT, FQ, 8>(lds, jb, je, xi, yi, zi, sx, sy, sz);
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                Sx[k] = sx[k] * cs;
                Sy[k] = sy[k] * cs;
                Sz[k] = sz[k] * cs;
            }
        } else {
            FF t[TPT];
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                const MixedSrc me = lds[il[k]];
                t[k].xh = me.xh;
                t[k].yh = me.yh;
                t[k].zh = me.zh;
                t[k].xl = me.xl;
                t[k].yl = me.yl;
                t[k].zl = me.zl;
            }
            float sx[TPT], sy[TPT], sz[TPT], cx[TPT], cy[TPT], cz[TPT];
#pragma unroll
            for (int k = 0; k < TPT; ++k) sx[k] = sy[k] = sz[k] = cx[k] = cy[k] = cz[k] = 0.0f;
            // sources four at a time, then the last one to three
            const int j4 = jb + ((je - jb) & ~3);
            for (int j = jb; j < j4; j += 4) {
#pragma unroll
                for (int uu = 0; uu < 4; ++uu) {
                    const MixedSrc q = lds[j + uu];
#pragma unroll
                    for (int k = 0; k < TPT; ++k) {
                        float tx, ty, tz;
                        pair_f32_terms<FQ>(q, t[k], tx, ty, tz);
                        kahan_add(tx, sx[k], cx[k]);
                        kahan_add(ty, sy[k], cy[k]);
                        kahan_add(tz, sz[k], cz[k]);
                    }
                }
            }
            for (int j = j4; j < je; ++j) {
                const MixedSrc q = lds[j];
#pragma unroll
                for (int k = 0; k < TPT; ++k) {
                    float tx, ty, tz;
                    pair_f32_terms<FQ>(q, t[k], tx, ty, tz);
                    kahan_add(tx, sx[k], cx[k]);
                    kahan_add(ty, sy[k], cy[k]);
                    kahan_add(tz, sz[k], cz[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < TPT; ++k) {
                Sx[k] = ((double)sx[k] - (double)cx[k]) * cs;
                Sy[k] = ((double)sy[k] - (double)cy[k]) * cs;
                Sz[k] = ((double)sz[k] - (double)cz[k]) * cs;
            }
        }
    }
}

template <int PREC, int BLOCK, bool X>
__global__ __launch_bounds__(BLOCK) void k_batch(double4* __restrict__ src,
                                                 double* __restrict__ vx,
                                                 double* __restrict__ vy,
                                                 double* __restrict__ vz,
                                                 double* __restrict__ ax,
                                                 double* __restrict__ ay,
                                                 double* __restrict__ az,
                                                 const double* __restrict__ qm,
                                                 const double* __restrict__ qe,
                                                 const double* __restrict__ mass,
                                                 const int32_t* __restrict__ species,
                                                 const TrapDev* __restrict__ traps,
                                                 const CoolDev* __restrict__ cool,
                                                 const int64_t* __restrict__ offsets,
                                                 const int32_t* __restrict__ order,
                                                 const int64_t* __restrict__ counter,
                                                 double* __restrict__ vacc,
                                                 double* __restrict__ vavg, int64_t n_pad,
                                                 int nsteps, int accel_only, double uq,
                                                 int tpt_req) {
    // ions per owner thread at most (a 64-thread block takes traps of <= 64 ions only)
    constexpr int KMAX = BLOCK >= 256 ? kMaxTrap / BLOCK : 1;
    // pair work of larger traps: TPT targets per thread read each source once
    // (at most 2 with 1024 threads, whose 128-VGPR budget 4 targets overflow)
    constexpr int TMAX = BLOCK >= 1024 ? 2 : 4;
    // uq != 0: every ion carries the charge uq (units of e); the pair sums then
    // run over r^-3 d alone and are scaled by the charge once.
    const bool fq = uq != 0.0 && batch_fq_on(PREC);
    using S = typename BatchSrc<PREC>::T;
    // the trap's source stream, sized at launch for the batch's largest trap
    static_assert(sizeof(S) == sizeof(double4), "source records of 32 bytes");
    extern __shared__ double4 lds_stream[];
    S* lds = reinterpret_cast<S*>(lds_stream);
    // partial sums of every (component, target k, thread): one barrier per step
    __shared__ double red[3 * TMAX * BLOCK];
    // cos(Omega t) of kRf consecutive steps, computed one step per thread ahead of
    // them (off the steps' dependent chain); two buffers, so that a refill never
    // meets a read of the steps before
    constexpr int kRf = 64;
    __shared__ double rf[2][kRf];

    const int tr = order[blockIdx.x];
    const int64_t o = offsets[tr];
    const int m = (int)(offsets[tr + 1] - o);
    const int m16 = (m + 15) & ~15;
    // owner slots: whole waves, except for traps of <= 64 ions, whose m owners
    // are followed by source parts of about four sources each (at most 8 parts:
    // the owners add the part sums in a dependent chain)
    const bool tiny = m <= 64;
    const int IS = tiny ? max(m, 1) : min((m + 63) & ~63, BLOCK);
    const int JP = tiny ? max(1, min(min(BLOCK / IS, (m + 3) / 4), 8)) : BLOCK / IS;
    const int tid = threadIdx.x;
    const int slot = tid % IS;
    const int jpart = tid / IS;
    const bool active = jpart < JP;
    const bool owner = jpart == 0;
    // sources per part when each thread has one target: whole FP32 runs of 8 in
    // the FP32 + FP64 mode, multiples of 4 otherwise (padding beyond m adds
    // nothing), so that the sources of a small trap spread over the parts; for
    // traps of <= 64 ions any count, so that a part's dependent chain stays short
    const int kGran = tiny ? 1 : (PREC == 1 ? 8 : 4);
    const int send = tiny ? m : (PREC == 1 ? m16 : (m + 3) & ~3);
    const int jlen = ((send + JP - 1) / JP + kGran - 1) / kGran * kGran;
    const int jb = min(jpart * jlen, send);
    const int je = min(jb + jlen, send);
    const TrapDev T = traps[tr];
    const int64_t k0 = *counter;
    // a lone trap (the small-trap path) is latency-bound: one target per thread
    // below kBatchTpt4 ions saves the extra reduction rounds
    const int tpt2_from = gridDim.x == 1 ? kBatchTpt4 : kBatchTpt2;
    int TPT = m >= kBatchTpt4 ? TMAX : (m >= tpt2_from ? 2 : 1);
    // a requested count (launch-shape tuning) for traps of kBatchTpt2 ions or more
    if (tpt_req > 0 && m >= kBatchTpt2) TPT = min(tpt_req, TMAX);
    // with several targets per thread, at least enough of them for the BLOCK
    // threads to cover the trap (TMAX * BLOCK >= kMaxTrap); one target per
    // thread covers any trap through the KMAX owner slots
    if (TPT > 1)
        while (TPT < TMAX && TPT * BLOCK < m) TPT *= 2;
    const int WS = ((m + 64 * TPT - 1) / (64 * TPT)) * 64;  // <= BLOCK
    const int JPW = BLOCK / WS;
    const int wslot = tid % WS, wpart = tid / WS;
    const bool wactive = wpart < JPW;
    const int wlen = ((m16 / JPW) + 15) & ~15;
    const int wjb = min(wpart * wlen, m16);
    const int wje = min(wjb + wlen, m16);

    double x[KMAX], y[KMAX], z[KMAX], u[KMAX], v[KMAX], w[KMAX], a0[KMAX], a1[KMAX], a2[KMAX];
    double q_m[KMAX], q_e[KMAX], m_i[KMAX];
    int32_t sp[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int il = slot + IS * k;
        if (owner && il < m) {
            const double4 p = src[o + il];
            x[k] = p.x;
            y[k] = p.y;
            z[k] = p.z;
            u[k] = vx[o + il];
            v[k] = vy[o + il];
            w[k] = vz[o + il];
            a0[k] = ax[o + il];
            a1[k] = ay[o + il];
            a2[k] = az[o + il];
            q_m[k] = qm[o + il];
            q_e[k] = qe[o + il];
            m_i[k] = mass[o + il];
            sp[k] = species[o + il];
        } else {
            x[k] = y[k] = z[k] = u[k] = v[k] = w[k] = a0[k] = a1[k] = a2[k] = 0.0;
            q_m[k] = q_e[k] = 0.0;
            m_i[k] = 1.0;
            sp[k] = 0;
        }
    }
    // the source ranges stop at m: no padding source is ever read
    const int jr0 = min(jb, m), jr1 = min(je, m);
    const int wjr0 = min(wjb, m), wjr1 = min(wje, m);

    const int total = accel_only ? 1 : nsteps;
    const int64_t step0 = cool->step_base + k0 + 1;  // run-wide number of the first step
    const CoolRef cr = cool_switches<X>(cool);
    for (int step = 0; step < total; ++step) {
        if (step % kRf == 0 && T.ps == 0.0 && tid < kRf && step + tid < total) {
            // read after the barrier below
            const int sq = step + tid;
            const double tq = T.t_start + (double)(k0 + sq + (accel_only ? 0 : 1)) * T.dt;
            rf[(step / kRf) & 1][tid] = cos(T.omega * tq);
        }
        // first half of the step; positions into the LDS source stream
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int il = slot + IS * k;
            if (owner && il < m) {
                if (!accel_only)
                    half_step_drift(T, cr, o + il, sp[k], m_i[k], step0 + step, x[k], y[k],
                                    z[k], u[k], v[k], w[k], a0[k], a1[k], a2[k]);
                if constexpr (PREC == 0) {
                    lds[il] = make_double4(x[k], y[k], z[k], 1.5 * q_e[k]);
                } else if constexpr (PREC == 1) {
                    lds[il] = make_batch_src(x[k], y[k], z[k], q_e[k]);
                } else {
                    lds[il] = make_src(x[k], y[k], z[k], q_e[k]);
                }
            }
        }
        __syncthreads();
        double Sx[KMAX], Sy[KMAX], Sz[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) Sx[k] = Sy[k] = Sz[k] = 0.0;
        if (TPT > 1) {
            // TPT targets per thread, partial sums to the owners in part order
            double Wx[4], Wy[4], Wz[4];
            if (wactive) {
                if constexpr (TMAX >= 4) {
                    if (TPT == 4) {
                        if (fq)
                            batch_pairs_multi<PREC, 4, true>(lds, m, wslot, WS, wjr0, wjr1, uq, Wx, Wy, Wz);
                        else
                            batch_pairs_multi<PREC, 4, false>(lds, m, wslot, WS, wjr0, wjr1, uq, Wx, Wy, Wz);
                    } else if (fq) {
                        batch_pairs_multi<PREC, 2, true>(lds, m, wslot, WS, wjr0, wjr1, uq, Wx, Wy, Wz);
                    } else {
                        batch_pairs_multi<PREC, 2, false>(lds, m, wslot, WS, wjr0, wjr1, uq, Wx, Wy, Wz);
                    }
                } else if (fq) {
                    batch_pairs_multi<PREC, 2, true>(lds, m, wslot, WS, wjr0, wjr1, uq, Wx, Wy, Wz);
                } else {
                    batch_pairs_multi<PREC, 2, false>(lds, m, wslot, WS, wjr0, wjr1, uq, Wx, Wy, Wz);
                }
            }
            if (wactive) {
#pragma unroll
                for (int k = 0; k < TMAX; ++k) {
                    if (k >= TPT) break;
                    red[(0 * TMAX + k) * BLOCK + tid] = Wx[k];
                    red[(1 * TMAX + k) * BLOCK + tid] = Wy[k];
                    red[(2 * TMAX + k) * BLOCK + tid] = Wz[k];
                }
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < KMAX; ++kk) {
                const int il = slot + IS * kk;
                if (owner && il < m) {
                    const int k = il / WS, r = il - WS * k;
                    for (int pp = 0; pp < JPW; ++pp) {
                        Sx[kk] += red[(0 * TMAX + k) * BLOCK + pp * WS + r];
                        Sy[kk] += red[(1 * TMAX + k) * BLOCK + pp * WS + r];
                        Sz[kk] += red[(2 * TMAX + k) * BLOCK + pp * WS + r];
                    }
                }
            }
        }
        // pair field of this thread's targets over its source part (one target per thread)
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int il = slot + IS * k;
            if (TPT > 1 || !active || il >= m) continue;
            double W1x[4], W1y[4], W1z[4];
            if (fq)
                batch_pairs_multi<PREC, 1, true>(lds, m, il, IS, jr0, jr1, uq, W1x, W1y, W1z);
            else
                batch_pairs_multi<PREC, 1, false>(lds, m, il, IS, jr0, jr1, uq, W1x, W1y, W1z);
            Sx[k] = W1x[0];
            Sy[k] = W1y[0];
            Sz[k] = W1z[0];
        }
        if (JP > 1 && TPT == 1) {
            // deterministic reduction over source parts: owners add parts in order
            // (only KMAX == 1 can have JP > 1, since JP > 1 needs m <= BLOCK / 2)
            if (active && jpart > 0) {
                red[0 * TMAX * BLOCK + tid] = Sx[0];
                red[1 * TMAX * BLOCK + tid] = Sy[0];
                red[2 * TMAX * BLOCK + tid] = Sz[0];
            }
            __syncthreads();
            if (owner) {
                for (int p = 1; p < JP; ++p) {
                    Sx[0] += red[0 * TMAX * BLOCK + slot + p * IS];
                    Sy[0] += red[1 * TMAX * BLOCK + slot + p * IS];
                    Sz[0] += red[2 * TMAX * BLOCK + slot + p * IS];
                }
            }
        }
        // every thread is past the pair loops before the next step writes the
        // source stream: the reductions above had a barrier, else one here
        if (TPT == 1 && JP == 1) __syncthreads();
        const double crf = T.ps == 0.0 ? rf[(step / kRf) & 1][step % kRf] : 0.0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int il = slot + IS * k;
            if (owner && il < m) {
                trap_accel_c(T, crf, q_m[k], x[k], y[k], z[k], Sx[k], Sy[k], Sz[k], a0[k],
                             a1[k], a2[k]);
                if (!accel_only) {
                    end_kick(T, cr, o + il, sp[k], m_i[k], step0 + step, u[k], v[k], w[k],
                             a0[k], a1[k], a2[k]);
                    time_average(cr, o + il, n_pad, step0 + step, vacc, vavg, u[k], v[k],
                                 w[k]);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int il = slot + IS * k;
        if (owner && il < m) {
            src[o + il] = make_double4(x[k], y[k], z[k], 1.5 * q_e[k]);
            vx[o + il] = u[k];
            vy[o + il] = v[k];
            vz[o + il] = w[k];
            ax[o + il] = a0[k];
            ay[o + il] = a1[k];
            az[o + il] = a2[k];
        }
    }
}

// ------------------------------------------------- traps of <= 64 ions, one wave
//
// The batched step of traps of at most 64 ions on one wave, with the target
// state in registers and no workgroup machinery: lane l works for target
// l / P over source part l % P (P a power of two, at most 8, chosen per launch
// from the largest trap m_max with m_max P <= 64; see wave_parts), the parts
// of a target sit in consecutive lanes and their sums are added by
// a fixed xor butterfly (every lane of the group ends with the same sum), and
// the owner (part 0) ends the step.  The arithmetic per pair and per step is
// that of k_batch (the same pair terms, FP32 runs of at most 8 sources, the
// cos(Omega t) table, the same step numbering for the cooling draws); part p
// sums the sources p, p + P, ... in order, the parts are added by the
// butterfly.

template <int PREC, int P, int W, bool X>
__global__ __launch_bounds__(64 * W) void k_wave(double4* __restrict__ src,
                                             double* __restrict__ vx, double* __restrict__ vy,
                                             double* __restrict__ vz, double* __restrict__ ax,
                                             double* __restrict__ ay, double* __restrict__ az,
                                             const double* __restrict__ qm,
                                             const double* __restrict__ qe,
                                             const double* __restrict__ mass,
                                             const int32_t* __restrict__ species,
                                             const TrapDev* __restrict__ traps,
                                             const CoolDev* __restrict__ cool,
                                             const int64_t* __restrict__ offsets,
                                             const int32_t* __restrict__ order,
                                             const int64_t* __restrict__ counter,
                                             double* __restrict__ vacc,
                                             double* __restrict__ vavg, int64_t n_pad,
                                             int nsteps, int accel_only) {
    using S = typename BatchSrc<PREC>::T;
    constexpr int kSlots = 64 * W / P;  // targets per workgroup
    __shared__ S lds[kSlots];
    constexpr int kRf = 64;
    __shared__ double rf[2][kRf];
    const int tr = order[blockIdx.x];
    const int64_t o = offsets[tr];
    const int m = (int)(offsets[tr + 1] - o);  // <= kSlots (checked by the host)
    const int lane = threadIdx.x;
    const int ti = lane / P, part = lane - ti * P;
    const bool owner = part == 0 && ti < m;
    const TrapDev T = traps[tr];
    const int64_t k0 = *counter;
    const int64_t step0 = cool->step_base + k0 + 1;  // run-wide number of the first step
    const CoolRef cr = cool_switches<X>(cool);
    const int64_t ion = o + min(ti, m - 1);
    double x = 0.0, y = 0.0, z = 0.0, u = 0.0, v = 0.0, w = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0;
    double q_m = 0.0, q_e = 0.0, m_i = 1.0;
    int32_t sp = 0;
    if (owner) {
        const double4 p = src[ion];
        x = p.x;
        y = p.y;
        z = p.z;
        u = vx[ion];
        v = vy[ion];
        w = vz[ion];
        a0 = ax[ion];
        a1 = ay[ion];
        a2 = az[ion];
        q_m = qm[ion];
        q_e = qe[ion];
        m_i = mass[ion];
        sp = species[ion];
    }
    const int total = accel_only ? 1 : nsteps;
    for (int step = 0; step < total; ++step) {
        if (step % kRf == 0 && T.ps == 0.0 && lane < kRf && step + lane < total) {
            const double tq =
                T.t_start + (double)(k0 + step + lane + (accel_only ? 0 : 1)) * T.dt;
            rf[(step / kRf) & 1][lane] = cos(T.omega * tq);
        }
        if (owner) {
            if (!accel_only)
                half_step_drift(T, cr, ion, sp, m_i, step0 + step, x, y, z, u, v, w, a0, a1,
                                a2);
            if constexpr (PREC == 0) {
                lds[ti] = make_double4(x, y, z, 1.5 * q_e);
            } else if constexpr (PREC == 1) {
                lds[ti] = make_batch_src(x, y, z, q_e);
            } else {
                lds[ti] = make_src(x, y, z, q_e);
            }
        }
        __syncthreads();
        double Sx = 0.0, Sy = 0.0, Sz = 0.0;
        const S me = lds[min(ti, m - 1)];
        // part p takes the sources p, p + P, ...: the P parts of a target read P
        // consecutive records at a time (no LDS bank conflicts between them)
        if constexpr (PREC == 0) {
            for (int j = part; j < m; j += P) pair_f64(lds[j], me.x, me.y, me.z, Sx, Sy, Sz);
        } else if constexpr (PREC == 1) {
            // FP32 runs of at most 8 sources, flushed to FP64
            for (int j0 = part; j0 < m; j0 += 8 * P) {
                float fx = 0.0f, fy = 0.0f, fz = 0.0f;
                const int j1 = min(j0 + 8 * P, m);
                for (int j = j0; j < j1; j += P) {
                    float tx, ty, tz;
                    batch_pair_f32<false>(lds[j], me.x, me.y, me.z, tx, ty, tz);
                    fx += tx;
                    fy += ty;
                    fz += tz;
                }
                Sx += (double)fx;
                Sy += (double)fy;
                Sz += (double)fz;
            }
            Sx *= kMixedFieldScale;
            Sy *= kMixedFieldScale;
            Sz *= kMixedFieldScale;
        } else {
            const FF t{me.xh, me.yh, me.zh, me.xl, me.yl, me.zl};
            float sx = 0.0f, sy = 0.0f, sz = 0.0f, cx = 0.0f, cy = 0.0f, cz = 0.0f;
            for (int j = part; j < m; j += P) {
                float tx, ty, tz;
                pair_f32_terms<false>(lds[j], t, tx, ty, tz);
                kahan_add(tx, sx, cx);
                kahan_add(ty, sy, cy);
                kahan_add(tz, sz, cz);
            }
            Sx = ((double)sx - (double)cx) * kMixedFieldScale;
            Sy = ((double)sy - (double)cy) * kMixedFieldScale;
            Sz = ((double)sz - (double)cz) * kMixedFieldScale;
        }
        // the parts of a target: a fixed butterfly over its P consecutive lanes
#pragma unroll
        for (int d = P / 2; d >= 1; d >>= 1) {
            Sx += __shfl_xor(Sx, d);
            Sy += __shfl_xor(Sy, d);
            Sz += __shfl_xor(Sz, d);
        }
        if (owner) {
            const double crf = T.ps == 0.0 ? rf[(step / kRf) & 1][step % kRf] : 0.0;
            trap_accel_c(T, crf, q_m, x, y, z, Sx, Sy, Sz, a0, a1, a2);
            if (!accel_only) {
                end_kick(T, cr, ion, sp, m_i, step0 + step, u, v, w, a0, a1, a2);
                time_average(cr, ion, n_pad, step0 + step, vacc, vavg, u, v, w);
            }
        }
        // every lane is past its reads of the source stream and the cos table
        __syncthreads();
    }
    if (owner) {
        src[ion] = make_double4(x, y, z, 1.5 * q_e);
        vx[ion] = u;
        vy[ion] = v;
        vz[ion] = w;
        ax[ion] = a0;
        ay[ion] = a1;
        az[ion] = a2;
    }
}

// ------------------------------------------------------------ rigid bodies

__device__ __forceinline__ void quat_rot(const double q[4], double A[9]) {
#pragma clang fp contract(off)
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    A[0] = 1.0 - 2.0 * (y * y + z * z);
    A[1] = 2.0 * (x * y - w * z);
    A[2] = 2.0 * (x * z + w * y);
    A[3] = 2.0 * (x * y + w * z);
    A[4] = 1.0 - 2.0 * (x * x + z * z);
    A[5] = 2.0 * (y * z - w * x);
    A[6] = 2.0 * (x * z - w * y);
    A[7] = 2.0 * (y * z + w * x);
    A[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Angular velocity w = A diag(inv_i) A^T L for orientation q.
__device__ __forceinline__ void rigid_omega(const double q[4], const double inv_i[3],
                                            const double L[3], double w[3]) {
#pragma clang fp contract(off)
    double A[9], p[3];
    quat_rot(q, A);
    for (int k = 0; k < 3; ++k) p[k] = (A[k] * L[0] + A[3 + k] * L[1] + A[6 + k] * L[2]) * inv_i[k];
    for (int r = 0; r < 3; ++r) w[r] = A[3 * r] * p[0] + A[3 * r + 1] * p[1] + A[3 * r + 2] * p[2];
}

// Normalised Euler step q + s (0, w) q of dq/dt = (1/2) (0, w) q.
__device__ __forceinline__ void quat_euler_step(const double q[4], const double w[3], double s,
                                                double out[4]) {
#pragma clang fp contract(off)
    const double dw = -(w[0] * q[1] + w[1] * q[2] + w[2] * q[3]);
    const double dx = w[0] * q[0] + (w[1] * q[3] - w[2] * q[2]);
    const double dy = w[1] * q[0] + (w[2] * q[1] - w[0] * q[3]);
    const double dz = w[2] * q[0] + (w[0] * q[2] - w[1] * q[1]);
    const double r0 = q[0] + s * dw, r1 = q[1] + s * dx, r2 = q[2] + s * dy, r3 = q[3] + s * dz;
    const double nrm = sqrt(r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3);
    out[0] = r0 / nrm;
    out[1] = r1 / nrm;
    out[2] = r2 / nrm;
    out[3] = r3 / nrm;
}

// Orientation over dt with L fixed: Richardson extrapolation of one Euler
// step of dt and two of dt/2 (w re-evaluated at the midpoint orientation).
__device__ __forceinline__ void rigid_rotate(double q[4], const double L[3],
                                             const double inv_i[3], double dt) {
#pragma clang fp contract(off)
    double w0[3], w1[3], qf[4], qh[4], qh2[4];
    rigid_omega(q, inv_i, L, w0);
    quat_euler_step(q, w0, 0.5 * dt, qf);
    quat_euler_step(q, w0, 0.25 * dt, qh);
    rigid_omega(qh, inv_i, L, w1);
    quat_euler_step(qh, w1, 0.25 * dt, qh2);
    double r[4];
    for (int k = 0; k < 4; ++k) r[k] = 2.0 * qh2[k] - qf[k];
    const double nrm = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
    for (int k = 0; k < 4; ++k) q[k] = r[k] / nrm;
}

// Force and torque on each body from its members' accelerations (one
// workgroup per body, members strided over the threads, tree reduction in a
// fixed order).  With END, also the end of the step for the body: half kick,
// damping half-step, angular velocity, and the members' velocities (with
// their time averages).
template <bool END>
__global__ __launch_bounds__(256) void k_rigid_wrench(RigidDev* __restrict__ bodies,
                                                      const int32_t* __restrict__ rstart,
                                                      const int32_t* __restrict__ rmembers,
                                                      const double* __restrict__ dbody,
                                                      const double* __restrict__ ax,
                                                      const double* __restrict__ ay,
                                                      const double* __restrict__ az,
                                                      const double* __restrict__ mass,
                                                      double* __restrict__ vx,
                                                      double* __restrict__ vy,
                                                      double* __restrict__ vz,
                                                      const TrapDev* __restrict__ traps,
                                                      const CoolDev* __restrict__ cool,
                                                      const int64_t* __restrict__ counter,
                                                      double* __restrict__ vacc,
                                                      double* __restrict__ vavg, int64_t n_pad) {
#pragma clang fp contract(off)
    __shared__ double red[6][256];
    __shared__ double shared_state[9];  // V, w, (pad)
    const int b = blockIdx.x, tid = threadIdx.x;
    RigidDev* B = bodies + b;
    double q[4] = {B->q[0], B->q[1], B->q[2], B->q[3]};
    double A[9];
    quat_rot(q, A);
    const int m0 = rstart[b], m1 = rstart[b + 1];
    double f[6] = {0, 0, 0, 0, 0, 0};
    for (int m = m0 + tid; m < m1; m += 256) {
        const int i = rmembers[m];
        const double d0 = dbody[i], d1 = dbody[n_pad + i], d2 = dbody[2 * n_pad + i];
        const double o0 = A[0] * d0 + A[1] * d1 + A[2] * d2;
        const double o1 = A[3] * d0 + A[4] * d1 + A[5] * d2;
        const double o2 = A[6] * d0 + A[7] * d1 + A[8] * d2;
        const double fx = mass[i] * ax[i], fy = mass[i] * ay[i], fz = mass[i] * az[i];
        f[0] += fx;
        f[1] += fy;
        f[2] += fz;
        f[3] += o1 * fz - o2 * fy;
        f[4] += o2 * fx - o0 * fz;
        f[5] += o0 * fy - o1 * fx;
    }
    for (int c = 0; c < 6; ++c) red[c][tid] = f[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w)
            for (int c = 0; c < 6; ++c) red[c][tid] += red[c][tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        double F[3] = {red[0][0], red[1][0], red[2][0]}, Tq[3] = {red[3][0], red[4][0], red[5][0]};
        for (int c = 0; c < 3; ++c) {
            B->F[c] = F[c];
            B->T[c] = Tq[c];
        }
        if (END) {
            const TrapDev T = traps[0];
            double V[3], L[3], w[3];
            for (int c = 0; c < 3; ++c) {
                V[c] = B->V[c] + T.h * (F[c] / B->M);
                L[c] = B->L[c] + T.h * Tq[c];
                V[c] = T.f * V[c];
                L[c] = T.f * L[c];
            }
            const double inv_i[3] = {B->inv_i[0], B->inv_i[1], B->inv_i[2]};
            rigid_omega(q, inv_i, L, w);
            for (int c = 0; c < 3; ++c) {
                B->V[c] = V[c];
                B->L[c] = L[c];
                B->w[c] = w[c];
                shared_state[c] = V[c];
                shared_state[3 + c] = w[c];
            }
        }
    }
    if (!END) return;
    __syncthreads();
    const double V0 = shared_state[0], V1 = shared_state[1], V2 = shared_state[2];
    const double w0 = shared_state[3], w1 = shared_state[4], w2 = shared_state[5];
    const int64_t step = cool->step_base + *counter;
    for (int m = m0 + tid; m < m1; m += 256) {
        const int i = rmembers[m];
        const double d0 = dbody[i], d1 = dbody[n_pad + i], d2 = dbody[2 * n_pad + i];
        const double o0 = A[0] * d0 + A[1] * d1 + A[2] * d2;
        const double o1 = A[3] * d0 + A[4] * d1 + A[5] * d2;
        const double o2 = A[6] * d0 + A[7] * d1 + A[8] * d2;
        const double u = V0 + (w1 * o2 - w2 * o1);
        const double v = V1 + (w2 * o0 - w0 * o2);
        const double w = V2 + (w0 * o1 - w1 * o0);
        vx[i] = u;
        vy[i] = v;
        vz[i] = w;
        time_average(load_cool(cool), i, n_pad, step, vacc, vavg, u, v, w);
    }
}

// First half of a step for each body: damping half-step, half kick, COM drift
// and the orientation update (one thread per body).
__global__ __launch_bounds__(64) void k_rigid_drift(RigidDev* __restrict__ bodies, int nbodies,
                                                    const TrapDev* __restrict__ traps) {
#pragma clang fp contract(off)
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbodies) return;
    const TrapDev T = traps[0];
    RigidDev* B = bodies + b;
    double V[3], L[3], R[3], q[4] = {B->q[0], B->q[1], B->q[2], B->q[3]};
    const double inv_i[3] = {B->inv_i[0], B->inv_i[1], B->inv_i[2]};
    for (int c = 0; c < 3; ++c) {
        V[c] = T.f * B->V[c];
        L[c] = T.f * B->L[c];
        V[c] = V[c] + T.h * (B->F[c] / B->M);
        L[c] = L[c] + T.h * B->T[c];
        R[c] = B->R[c] + T.dt * V[c];
    }
    rigid_rotate(q, L, inv_i, T.dt);
    double w[3];
    rigid_omega(q, inv_i, L, w);
    for (int c = 0; c < 3; ++c) {
        B->V[c] = V[c];
        B->L[c] = L[c];
        B->R[c] = R[c];
        B->w[c] = w[c];
    }
    for (int k = 0; k < 4; ++k) B->q[k] = q[k];
}

// Members placed at R + A(q) d (positions and both source streams).
__global__ __launch_bounds__(256) void k_rigid_place(const RigidDev* __restrict__ bodies,
                                                     const int32_t* __restrict__ rb,
                                                     const double* __restrict__ dbody,
                                                     double4* __restrict__ src,
                                                     MixedSrc* __restrict__ srcm,
                                                     const double* __restrict__ qe, int64_t n,
                                                     int64_t n_pad) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = rb[i];
    if (b < 0) return;
    const RigidDev* B = bodies + b;
    const double q[4] = {B->q[0], B->q[1], B->q[2], B->q[3]};
    double A[9];
    quat_rot(q, A);
    const double d0 = dbody[i], d1 = dbody[n_pad + i], d2 = dbody[2 * n_pad + i];
    const double x = B->R[0] + (A[0] * d0 + A[1] * d1 + A[2] * d2);
    const double y = B->R[1] + (A[3] * d0 + A[4] * d1 + A[5] * d2);
    const double z = B->R[2] + (A[6] * d0 + A[7] * d1 + A[8] * d2);
    double4 p = src[i];
    p.x = x;
    p.y = y;
    p.z = z;
    src[i] = p;
    if (srcm) srcm[i] = make_src(x, y, z, qe[i]);
}

// ------------------------------------------------------------ minimisation

// Per block of 256 ions: sums of v.F and F.F and the largest |F| (F = M a),
// reduced over the block in a fixed tree order.
__global__ __launch_bounds__(256) void k_min_partial(const double* __restrict__ vx,
                                                     const double* __restrict__ vy,
                                                     const double* __restrict__ vz,
                                                     const double* __restrict__ ax,
                                                     const double* __restrict__ ay,
                                                     const double* __restrict__ az,
                                                     const double* __restrict__ mass, int64_t n,
                                                     double* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double r[3][256];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 256 + tid;
    double P = 0.0, FF = 0.0, fm = 0.0;
    if (i < n) {
        const double fx = mass[i] * ax[i], fy = mass[i] * ay[i], fz = mass[i] * az[i];
        P = vx[i] * fx + vy[i] * fy + vz[i] * fz;
        FF = fx * fx + fy * fy + fz * fz;
        fm = sqrt(FF);
    }
    r[0][tid] = P;
    r[1][tid] = FF;
    r[2][tid] = fm;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            r[0][tid] += r[0][tid + w];
            r[1][tid] += r[1][tid + w];
            r[2][tid] = fmax(r[2][tid], r[2][tid + w]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        part[3 * blockIdx.x] = r[0][0];
        part[3 * blockIdx.x + 1] = r[1][0];
        part[3 * blockIdx.x + 2] = r[2][0];
    }
}

// One block: the partials in a fixed order, then the stopping test.
__global__ __launch_bounds__(256) void k_min_final(const double* __restrict__ part, int nblocks,
                                                   MinDev* __restrict__ ms) {
#pragma clang fp contract(off)
    __shared__ double r[3][256];
    const int tid = threadIdx.x;
    double P = 0.0, FF = 0.0, fm = 0.0;
    for (int b = tid; b < nblocks; b += 256) {
        P += part[3 * b];
        FF += part[3 * b + 1];
        fm = fmax(fm, part[3 * b + 2]);
    }
    r[0][tid] = P;
    r[1][tid] = FF;
    r[2][tid] = fm;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            r[0][tid] += r[0][tid + w];
            r[1][tid] += r[1][tid + w];
            r[2][tid] = fmax(r[2][tid], r[2][tid + w]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        ms->P = r[0][0];
        ms->FF = r[1][0];
        ms->fmax = r[2][0];
        ms->done = (r[2][0] <= ms->ftol || ms->iterations >= ms->max_iter) ? 1 : 0;
    }
}

// One iteration's move: keep the velocity's component along the 3N force (or
// drop it), kick by dt a, cap each ion's move at dmax, drift.  Does nothing
// once the stopping test has passed.
__global__ __launch_bounds__(256) void k_min_move(double4* __restrict__ src,
                                                  MixedSrc* __restrict__ srcm,
                                                  double* __restrict__ vx,
                                                  double* __restrict__ vy,
                                                  double* __restrict__ vz,
                                                  const double* __restrict__ ax,
                                                  const double* __restrict__ ay,
                                                  const double* __restrict__ az,
                                                  const double* __restrict__ mass,
                                                  const double* __restrict__ qe, int64_t n,
                                                  MinDev* __restrict__ ms) {
#pragma clang fp contract(off)
    if (ms->done) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double dt = ms->dt, dmax = ms->dmax, P = ms->P, FF = ms->FF;
    if (i == 0) ms->iterations += 1;  // one thread; nobody else reads it in this launch
    if (i >= n) return;
    const double coef = (P > 0.0 && FF > 0.0) ? P / FF : 0.0;
    double u = coef * (mass[i] * ax[i]), v = coef * (mass[i] * ay[i]), w = coef * (mass[i] * az[i]);
    u = u + dt * ax[i];
    v = v + dt * ay[i];
    w = w + dt * az[i];
    const double step = dt * sqrt(u * u + v * v + w * w);
    if (step > dmax) {
        const double r = dmax / step;
        u = u * r;
        v = v * r;
        w = w * r;
    }
    vx[i] = u;
    vy[i] = v;
    vz[i] = w;
    double4 p = src[i];
    p.x = p.x + dt * u;
    p.y = p.y + dt * v;
    p.z = p.z + dt * w;
    src[i] = p;
    if (srcm) srcm[i] = make_src(p.x, p.y, p.z, qe[i]);
}

// ------------------------------------------------------------ normal modes

// Mass-weighted Hessian of the static potential, one 3x3 block (i, j) per
// thread, written row-major into D (3n x 3n).  Off-diagonal blocks:
// k_e Q_i Q_j (delta/r^3 - 3 r r^T / r^5) / sqrt(M_i M_j), r = x_i - x_j.
// Diagonal blocks: minus the sum of those over j (ascending j), plus the trap
// curvature (pseudopotential and dc), divided by M_i.
__global__ __launch_bounds__(256) void k_hessian(const double4* __restrict__ src,
                                                 const double* __restrict__ qe,
                                                 const double* __restrict__ mass, int64_t n,
                                                 TrapDev T, double* __restrict__ D) {
#pragma clang fp contract(off)
    const int64_t j = (int64_t)blockIdx.x * 16 + threadIdx.x % 16;
    const int64_t i = (int64_t)blockIdx.y * 16 + threadIdx.x / 16;
    if (i >= n || j >= n) return;
    const int64_t m = 3 * n;
    const double ke = 1.0 / (4.0 * kPi * kEps0);
    const double4 pi = src[i];
    const double Qi = qe[i] * kElementaryCharge;
    if (i != j) {
        const double4 pj = src[j];
        const double r[3] = {pi.x - pj.x, pi.y - pj.y, pi.z - pj.z};
        const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double w = 1.0 / sqrt(mass[i] * mass[j]);
        double inv_r3 = 0.0, inv_r5 = 0.0, c = 0.0;
        if (r2 != 0.0) {
            const double inv_r = 1.0 / sqrt(r2);
            inv_r3 = inv_r * inv_r * inv_r;
            inv_r5 = inv_r3 * inv_r * inv_r;
            c = ke * Qi * (qe[j] * kElementaryCharge);
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                D[(3 * i + a) * m + 3 * j + b] =
                    c * ((a == b ? inv_r3 : 0.0) - 3.0 * r[a] * r[b] * inv_r5) * w;
        return;
    }
    double diag[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int64_t k = 0; k < n; ++k) {
        if (k == i) continue;
        const double4 pk = src[k];
        const double r[3] = {pi.x - pk.x, pi.y - pk.y, pi.z - pk.z};
        const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (r2 == 0.0) continue;
        const double inv_r = 1.0 / sqrt(r2);
        const double inv_r3 = inv_r * inv_r * inv_r, inv_r5 = inv_r3 * inv_r * inv_r;
        const double c = ke * Qi * (qe[k] * kElementaryCharge);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                diag[a][b] -= c * ((a == b ? inv_r3 : 0.0) - 3.0 * r[a] * r[b] * inv_r5);
    }
    const double qm = Qi / mass[i];
    diag[0][0] += Qi * qm * T.ps - Qi * T.a_dc;
    diag[1][1] += Qi * qm * T.ps - Qi * T.a_dc;
    diag[2][2] += 2.0 * Qi * T.a_dc;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) D[(3 * i + a) * m + 3 * i + b] = diag[a][b] / mass[i];
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

inline int n64_of(int64_t n) { return (int)((n + 63) & ~int64_t(63)); }

inline BodyMask body_mask(const DevState& s) {
    BodyMask m;
    m.code = s.body_code;
    m.gmin = s.body_gmin;
    m.gmax = s.body_gmax;
    return m;
}

template <int I>
hipError_t pair_f64_launch(const DevState& s, const LaunchShape& ls, int64_t* ctr,
                           hipStream_t st) {
    dim3 grid(blocks_for(s.n, 64 * I), ls.j_split);
    k_pair_f64<I><<<grid, 256, 0, st>>>(s.src, s.n, n64_of(s.n), ls.jps, s.n_pad, s.part, ctr,
                                         body_mask(s));
    return hipGetLastError();
}

template <int I, int L, bool KAHAN>
hipError_t pair_mixed_launch(const DevState& s, const LaunchShape& ls, int64_t* ctr,
                             hipStream_t st) {
    dim3 grid(blocks_for(s.n, 64 * I), ls.j_split);
    if (ls.lds_sources)
        k_pair_mixed_l<I, L, KAHAN><<<grid, 256, 0, st>>>(s.srcm, s.n, n64_of(s.n), ls.jps,
                                                          s.n_pad, s.part, ctr, body_mask(s));
    else
        k_pair_mixed_s<I, L, KAHAN><<<grid, 256, 0, st>>>(s.srcm, s.n, n64_of(s.n), ls.jps,
                                                          s.n_pad, s.part, ctr, body_mask(s));
    return hipGetLastError();
}

template <int I>
hipError_t pair_mixed_dispatch_l(const DevState& s, const LaunchShape& ls, int64_t* ctr,
                                 hipStream_t st) {
    switch (ls.flush_len) {
        case 4: return pair_mixed_launch<I, 4, false>(s, ls, ctr, st);
        case 16: return pair_mixed_launch<I, 16, false>(s, ls, ctr, st);
        default: return pair_mixed_launch<I, 8, false>(s, ls, ctr, st);
    }
}

template <int PREC, int BLOCK, bool X>
hipError_t batch_launch(const DevState& s, int n_traps, int max_trap, int nsteps,
                        int accel_only, double uq, int tpt, hipStream_t st) {
    const size_t stream_bytes = (size_t)max_trap * sizeof(double4);
    k_batch<PREC, BLOCK, X><<<n_traps, BLOCK, stream_bytes, st>>>(s.src, s.vx, s.vy, s.vz, s.ax, s.ay,
                                                       s.az, s.qm, s.qe, s.mass, s.species,
                                                       s.traps, s.cool, s.offsets, s.order,
                                                       s.counter, s.vacc, s.vavg, s.n_pad,
                                                       nsteps, accel_only, uq, tpt);
    return hipGetLastError();
}

template <int PREC, int P, int W, bool X>
hipError_t wave_launch_p(const DevState& s, int n_traps, int nsteps, int accel_only,
                         hipStream_t st) {
    k_wave<PREC, P, W, X><<<n_traps, 64 * W, 0, st>>>(s.src, s.vx, s.vy, s.vz, s.ax, s.ay, s.az,
                                                      s.qm, s.qe, s.mass, s.species, s.traps,
                                                      s.cool, s.offsets, s.order, s.counter,
                                                      s.vacc, s.vavg, s.n_pad, nsteps,
                                                      accel_only);
    return hipGetLastError();
}

// Parts per target of the one-wave kernel for traps of at most max_trap ions: a
// power of two, at most 8 and at most the trap size, with max_trap * P <= 64
// (8 ions: 8 parts of one source, 0.41 against 0.57 us per step with 2 parts of
// four in a stand-alone loop; 2 ions: 2 parts, 0.32 against 0.49 with 32).
inline int wave_parts(int max_trap) {
    int P = 1;
    while (P < 8 && 2 * P <= max_trap && 2 * P * max_trap <= 64) P *= 2;
    return P;
}

template <int PREC, bool X>
hipError_t wave_launch(const DevState& s, int n_traps, int max_trap, int nsteps, int accel_only,
                       hipStream_t st) {
    switch (wave_parts(max_trap)) {
        case 8: return wave_launch_p<PREC, 8, 1, X>(s, n_traps, nsteps, accel_only, st);
        case 4: return wave_launch_p<PREC, 4, 1, X>(s, n_traps, nsteps, accel_only, st);
        case 2: return wave_launch_p<PREC, 2, 1, X>(s, n_traps, nsteps, accel_only, st);
        default: return wave_launch_p<PREC, 1, 1, X>(s, n_traps, nsteps, accel_only, st);
    }
}

// The same kernel on block / 64 waves with 8 parts per target, for traps of at
// most block / 8 ions (a target's parts stay within one wave).
constexpr int kWaveMultiIons = 48;
template <int PREC, bool X>
hipError_t wave_launch_multi(const DevState& s, int n_traps, int block, int nsteps,
                             int accel_only, hipStream_t st) {
    switch (block) {
        case 1024: return wave_launch_p<PREC, 8, 16, X>(s, n_traps, nsteps, accel_only, st);
        case 512: return wave_launch_p<PREC, 8, 8, X>(s, n_traps, nsteps, accel_only, st);
        default: return wave_launch_p<PREC, 8, 4, X>(s, n_traps, nsteps, accel_only, st);
    }
}

template <int PREC, bool X>
hipError_t batch_dispatch_x(const DevState& s, int n_traps, int max_trap, int block, int nsteps,
                            int accel_only, double uq, int tpt, hipStream_t st) {
    // traps of at most 48 ions and block / 8: the wave kernel on block / 64 waves
    // (us per step FP64 / FP32 pairs against the batched kernel: 20 ions 0.88 / 0.99
    // against 1.15 / 1.30, 32 ions 1.02 / 1.13 against 1.32 / 1.48, 48 ions 1.31 /
    // 1.39 against 1.50 / 1.49; 64 ions 1.64 / 1.63 against 1.63 / 1.52 and 100
    // ions 3.29 / 3.03 against 2.72 / 2.35, so larger traps keep the batched kernel)
    if (block != 64 && 8 * max_trap <= block && max_trap <= kWaveMultiIons)
        return wave_launch_multi<PREC, X>(s, n_traps, block, nsteps, accel_only, st);
    switch (block) {
        case 64: return wave_launch<PREC, X>(s, n_traps, max_trap, nsteps, accel_only, st);
        case 512: return batch_launch<PREC, 512, X>(s, n_traps, max_trap, nsteps, accel_only, uq, tpt, st);
        case 1024: return batch_launch<PREC, 1024, X>(s, n_traps, max_trap, nsteps, accel_only, uq, tpt, st);
        default: return batch_launch<PREC, 256, X>(s, n_traps, max_trap, nsteps, accel_only, uq, tpt, st);
    }
}

template <int PREC>
hipError_t batch_dispatch(const DevState& s, int n_traps, int max_trap, int block, int nsteps, int accel_only,
                          bool cool_on, double uq, int tpt, hipStream_t st) {
    return cool_on ? batch_dispatch_x<PREC, true>(s, n_traps, max_trap, block, nsteps, accel_only, uq, tpt, st)
                   : batch_dispatch_x<PREC, false>(s, n_traps, max_trap, block, nsteps, accel_only, uq, tpt, st);
}

}  // namespace

hipError_t launch_drift(const DevState& s, bool cool_on, hipStream_t st) {
    if (cool_on)
        k_drift<true><<<blocks_for(s.n, 256), 256, 0, st>>>(
            s.src, s.srcm, s.vx, s.vy, s.vz, s.ax, s.ay, s.az, s.qe, s.mass, s.species, s.traps,
            s.cool, s.counter, s.rb, s.n);
    else
        k_drift<false><<<blocks_for(s.n, 256), 256, 0, st>>>(
            s.src, s.srcm, s.vx, s.vy, s.vz, s.ax, s.ay, s.az, s.qe, s.mass, s.species, s.traps,
            s.cool, s.counter, s.rb, s.n);
    return hipGetLastError();
}

hipError_t launch_pack_inputs(const double* x, const double* y, const double* z,
                              const double* charge, const double* mass, const DevState& s,
                              const TrapDev& T, hipStream_t st) {
    k_pack_inputs<<<blocks_for(s.n_pad, 256), 256, 0, st>>>(x, y, z, charge, mass, s.n, s.n_pad,
                                                            s.src, s.srcm, s.qm, s.qe, T,
                                                            s.traps);
    return hipGetLastError();
}

hipError_t launch_pack_mixed(const DevState& s, hipStream_t st) {
    if (!s.srcm) return hipSuccess;
    k_pack_mixed<<<blocks_for(s.n_pad, 256), 256, 0, st>>>(s.src, s.srcm, s.qe, s.n, s.n_pad);
    return hipGetLastError();
}

hipError_t launch_pair(const DevState& s, int precision, const LaunchShape& ls, bool count_step,
                       hipStream_t st) {
    int64_t* ctr = count_step ? s.counter : nullptr;
    if (ls.symmetric) {
        const int nb = sym_tiles(s.n);
        const unsigned units = (unsigned)(nb * (nb + 1) / 2);
        const double uq = ls.uniform_q;                // 0: charges differ
        const int full = (int)(s.n / kSymTile);        // tiles without padding
        const int32_t* tb = s.body_code ? s.tile_body : nullptr;  // exclusion by whole tiles
        const BodyTiles bt{s.body_code, s.tile_bmin, s.tile_bmax};
        if (precision == 2) {
            // the compensated mode: the built-in FP32 shape with Kahan sums
            if (ls.sym_masked)
                k_pair_mixed_sym<8, 8, 4, 2, true, true, true><<<units, 256, 0, st>>>(
                    s.srcm, s.n, nb, s.n_pad, s.part, ctr, (float)uq, full, tb, bt);
            else
                k_pair_mixed_sym<8, 8, 4, 2, true, false, true><<<units, 256, 0, st>>>(
                    s.srcm, s.n, nb, s.n_pad, s.part, ctr, (float)uq, full, tb);
            return hipGetLastError();
        }
        if (ls.sym_masked) {
            // bodies share tiles with other ions: the built-in variants with the per-pair test
            if (precision == 0)
                k_pair_f64_sym<4, 1, true, true><<<units, 256, 0, st>>>(
                    s.src, s.qe, s.n, nb, s.n_pad, s.part, ctr, uq, full, tb, bt);
            else
                k_pair_mixed_sym<8, 8, 4, 2, true, true><<<units, 256, 0, st>>>(
                    s.srcm, s.n, nb, s.n_pad, s.part, ctr, (float)uq, full, tb, bt);
            return hipGetLastError();
        }
        if (precision == 0) {
            switch (ls.sym_variant) {
                case 1:
                    k_pair_f64_sym<4, 1><<<units, 256, 0, st>>>(s.src, s.qe, s.n, nb, s.n_pad, s.part, ctr, uq, full, tb);
                    break;
                case 2:
                    k_pair_f64_sym<3, 1><<<units, 256, 0, st>>>(s.src, s.qe, s.n, nb, s.n_pad, s.part, ctr, uq, full, tb);
                    break;
                case 3:
                    k_pair_f64_sym<4, 2><<<units, 256, 0, st>>>(s.src, s.qe, s.n, nb, s.n_pad, s.part, ctr, uq, full, tb);
                    break;
                case 4:
                    k_pair_f64_sym<2, 2><<<units, 256, 0, st>>>(s.src, s.qe, s.n, nb, s.n_pad, s.part, ctr, uq, full, tb);
                    break;
                case 5:
                    k_pair_f64_sym<4, 1, true><<<units, 256, 0, st>>>(s.src, s.qe, s.n, nb, s.n_pad, s.part, ctr, uq, full, tb);
                    break;
                case 6:
                    k_pair_f64_sym<3, 2, true><<<units, 256, 0, st>>>(s.src, s.qe, s.n, nb, s.n_pad, s.part, ctr, uq, full, tb);
                    break;
                default:
                    k_pair_f64_sym<3, 2><<<units, 256, 0, st>>>(s.src, s.qe, s.n, nb, s.n_pad, s.part, ctr, uq, full, tb);
                    break;
            }
        } else {
            switch (ls.sym_variant) {
                case 1:
                    k_pair_mixed_sym<8, 4, 5, 1><<<units, 256, 0, st>>>(s.srcm, s.n, nb, s.n_pad, s.part, ctr, (float)uq, full, tb);
                    break;
                case 2:
                    k_pair_mixed_sym<8, 4, 6, 1><<<units, 256, 0, st>>>(s.srcm, s.n, nb, s.n_pad, s.part, ctr, (float)uq, full, tb);
                    break;
                case 3:
                    k_pair_mixed_sym<8, 8, 5, 1><<<units, 256, 0, st>>>(s.srcm, s.n, nb, s.n_pad, s.part, ctr, (float)uq, full, tb);
                    break;
                case 4:
                    k_pair_mixed_sym<8, 4, 4, 1><<<units, 256, 0, st>>>(s.srcm, s.n, nb, s.n_pad, s.part, ctr, (float)uq, full, tb);
                    break;
                case 5:
                    k_pair_mixed_sym<8, 8, 5, 1, true><<<units, 256, 0, st>>>(s.srcm, s.n, nb, s.n_pad, s.part, ctr, (float)uq, full, tb);
                    break;
                case 6:
                    k_pair_mixed_sym<8, 8, 4, 2, true><<<units, 256, 0, st>>>(s.srcm, s.n, nb, s.n_pad, s.part, ctr, (float)uq, full, tb);
                    break;
                case 7:  // the shape of 7 with FP32 runs of 16 sources
                    k_pair_mixed_sym<16, 8, 4, 2, true><<<units, 256, 0, st>>>(s.srcm, s.n, nb, s.n_pad, s.part, ctr, (float)uq, full, tb);
                    break;
                case 8:  // the shape of 7 with FP32 runs of 64 sources (a wave's share)
                    k_pair_mixed_sym<64, 8, 4, 2, true><<<units, 256, 0, st>>>(s.srcm, s.n, nb, s.n_pad, s.part, ctr, (float)uq, full, tb);
                    break;
                default:
                    k_pair_mixed_sym<8, 8, 4, 2><<<units, 256, 0, st>>>(s.srcm, s.n, nb, s.n_pad, s.part, ctr, (float)uq, full, tb);
                    break;
            }
        }
        return hipGetLastError();
    }
    if (precision == 0) {
        switch (ls.i_per_lane) {
            case 1: return pair_f64_launch<1>(s, ls, ctr, st);
            case 4: return pair_f64_launch<4>(s, ls, ctr, st);
            default: return pair_f64_launch<2>(s, ls, ctr, st);
        }
    }
    if (precision == 2) {
        switch (ls.i_per_lane) {
            case 1: return pair_mixed_launch<1, 8, true>(s, ls, ctr, st);
            case 4: return pair_mixed_launch<4, 8, true>(s, ls, ctr, st);
            default: return pair_mixed_launch<2, 8, true>(s, ls, ctr, st);
        }
    }
    switch (ls.i_per_lane) {
        case 1: return pair_mixed_dispatch_l<1>(s, ls, ctr, st);
        case 4: return pair_mixed_dispatch_l<4>(s, ls, ctr, st);
        default: return pair_mixed_dispatch_l<2>(s, ls, ctr, st);
    }
}

template <int MODE, int UW, typename PT>
void update_launch(const DevState& s, const LaunchShape& ls, double scale, MixedSrc* srcm,
                   const int64_t* ctr, hipStream_t st) {
    const unsigned g = blocks_for(s.n, 64);  // 64 ions per block of UW waves
    const PT* part = reinterpret_cast<const PT*>(s.part);
    if (ls.cool_on && MODE != kModeAccel)
        k_update<MODE, UW, true, PT><<<g, 64 * UW, 0, st>>>(
            s.src, srcm, s.vx, s.vy, s.vz, s.ax, s.ay, s.az, s.qm, s.qe, s.mass, s.species,
            part, ls.j_split, s.n, s.n_pad, scale, s.traps, s.cool, ctr, s.vacc, s.vavg, s.rb);
    else
        k_update<MODE, UW, false, PT><<<g, 64 * UW, 0, st>>>(
            s.src, srcm, s.vx, s.vy, s.vz, s.ax, s.ay, s.az, s.qm, s.qe, s.mass, s.species,
            part, ls.j_split, s.n, s.n_pad, scale, s.traps, s.cool, ctr, s.vacc, s.vavg, s.rb);
}

template <int MODE, typename PT>
void update_dispatch_t(const DevState& s, const LaunchShape& ls, double scale, MixedSrc* srcm,
                       const int64_t* ctr, hipStream_t st) {
    if (ls.update_waves == 16)
        update_launch<MODE, 16, PT>(s, ls, scale, srcm, ctr, st);
    else if (ls.update_waves == 8)
        update_launch<MODE, 8, PT>(s, ls, scale, srcm, ctr, st);
    else
        update_launch<MODE, 4, PT>(s, ls, scale, srcm, ctr, st);
}

// The pair kernels of the FP32 + FP64-run mode leave FP32 partials, those of
// the FP64 and compensated modes FP64 ones.
template <int MODE>
void update_dispatch(const DevState& s, const LaunchShape& ls, double scale, MixedSrc* srcm,
                     const int64_t* ctr, hipStream_t st, bool f32_partials) {
    if (f32_partials)
        update_dispatch_t<MODE, float>(s, ls, scale, srcm, ctr, st);
    else
        update_dispatch_t<MODE, double>(s, ls, scale, srcm, ctr, st);
}

hipError_t launch_update(const DevState& s, int precision, const LaunchShape& ls, int mode,
                         bool use_counter, hipStream_t st) {
    const double scale = precision == 0 ? 1.0 : kMixedFieldScale;
    const int64_t* ctr = use_counter ? s.counter : nullptr;
    MixedSrc* srcm = precision == 0 ? nullptr : s.srcm;
    const bool f32 = precision == 1;
    switch (mode) {
        case kModeAccel: update_dispatch<kModeAccel>(s, ls, scale, srcm, ctr, st, f32); break;
        case kModeEnd: update_dispatch<kModeEnd>(s, ls, scale, srcm, ctr, st, f32); break;
        default: update_dispatch<kModeEndDrift>(s, ls, scale, srcm, ctr, st, f32); break;
    }
    return hipGetLastError();
}

hipError_t launch_rigid_wrench(const DevState& s, bool end_kick, hipStream_t st) {
    if (s.nbodies <= 0) return hipSuccess;
    if (end_kick)
        k_rigid_wrench<true><<<s.nbodies, 256, 0, st>>>(s.rigid, s.rstart, s.rmembers, s.dbody,
                                                        s.ax, s.ay, s.az, s.mass, s.vx, s.vy,
                                                        s.vz, s.traps, s.cool, s.counter, s.vacc,
                                                        s.vavg, s.n_pad);
    else
        k_rigid_wrench<false><<<s.nbodies, 256, 0, st>>>(s.rigid, s.rstart, s.rmembers, s.dbody,
                                                         s.ax, s.ay, s.az, s.mass, s.vx, s.vy,
                                                         s.vz, s.traps, s.cool, s.counter,
                                                         s.vacc, s.vavg, s.n_pad);
    return hipGetLastError();
}

hipError_t launch_rigid_drift(const DevState& s, hipStream_t st) {
    if (s.nbodies <= 0) return hipSuccess;
    k_rigid_drift<<<blocks_for(s.nbodies, 64), 64, 0, st>>>(s.rigid, s.nbodies, s.traps);
    return hipGetLastError();
}

hipError_t launch_rigid_place(const DevState& s, int precision, hipStream_t st) {
    if (s.nbodies <= 0) return hipSuccess;
    MixedSrc* srcm = precision == 0 ? nullptr : s.srcm;
    k_rigid_place<<<blocks_for(s.n, 256), 256, 0, st>>>(s.rigid, s.rb, s.dbody, s.src, srcm, s.qe,
                                                        s.n, s.n_pad);
    return hipGetLastError();
}

hipError_t launch_min_reduce(const DevState& s, hipStream_t st) {
    const unsigned nb = blocks_for(s.n, 256);
    k_min_partial<<<nb, 256, 0, st>>>(s.vx, s.vy, s.vz, s.ax, s.ay, s.az, s.mass, s.n, s.minpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_min_final<<<1, 256, 0, st>>>(s.minpart, (int)nb, s.minst);
    return hipGetLastError();
}

hipError_t launch_min_move(const DevState& s, int precision, hipStream_t st) {
    MixedSrc* srcm = precision == 0 ? nullptr : s.srcm;
    k_min_move<<<blocks_for(s.n, 256), 256, 0, st>>>(s.src, srcm, s.vx, s.vy, s.vz, s.ax, s.ay,
                                                     s.az, s.mass, s.qe, s.n, s.minst);
    return hipGetLastError();
}

hipError_t launch_hessian(const DevState& s, const TrapDev& T, double* D, hipStream_t st) {
    const unsigned g = blocks_for(s.n, 16);
    k_hessian<<<dim3(g, g), 256, 0, st>>>(s.src, s.qe, s.mass, s.n, T, D);
    return hipGetLastError();
}

hipError_t launch_batch(const DevState& s, int precision, int n_traps, int max_trap,
                        const LaunchShape& ls, int nsteps, int, hipStream_t st) {
    switch (precision) {
        case 0: return batch_dispatch<0>(s, n_traps, max_trap, ls.batch_block, nsteps, 0, ls.cool_on, ls.uniform_q, ls.batch_tpt, st);
        case 2: return batch_dispatch<2>(s, n_traps, max_trap, ls.batch_block, nsteps, 0, ls.cool_on, ls.uniform_q, ls.batch_tpt, st);
        default: return batch_dispatch<1>(s, n_traps, max_trap, ls.batch_block, nsteps, 0, ls.cool_on, ls.uniform_q, ls.batch_tpt, st);
    }
}

hipError_t launch_batch_accel(const DevState& s, int precision, int n_traps, int max_trap,
                              const LaunchShape& ls, hipStream_t st) {
    switch (precision) {
        case 0: return batch_dispatch<0>(s, n_traps, max_trap, ls.batch_block, 0, 1, false, ls.uniform_q, ls.batch_tpt, st);
        case 2: return batch_dispatch<2>(s, n_traps, max_trap, ls.batch_block, 0, 1, false, ls.uniform_q, ls.batch_tpt, st);
        default: return batch_dispatch<1>(s, n_traps, max_trap, ls.batch_block, 0, 1, false, ls.uniform_q, ls.batch_tpt, st);
    }
}

namespace {

template <int PREC, int TR>
hipError_t rows_launch(const RowsArgs& A, bool cool_on, int mode, int k, hipStream_t st) {
    const unsigned g = (unsigned)((A.n + TR - 1) / TR);
    if (cool_on && mode != kModeAccel)
        k_rows<PREC, TR, true><<<g, kRowsBlock, 0, st>>>(A, mode, k);
    else
        k_rows<PREC, TR, false><<<g, kRowsBlock, 0, st>>>(A, mode, k);
    return hipGetLastError();
}

template <int PREC>
hipError_t rows_dispatch(const RowsArgs& A, int tr, bool cool_on, int mode, int k,
                         hipStream_t st) {
    switch (tr) {
        case 1: return rows_launch<PREC, 1>(A, cool_on, mode, k, st);
        case 2: return rows_launch<PREC, 2>(A, cool_on, mode, k, st);
        case 8: return rows_launch<PREC, 8>(A, cool_on, mode, k, st);
        default: return rows_launch<PREC, 4>(A, cool_on, mode, k, st);
    }
}

}  // namespace

hipError_t launch_rows(const DevState& s, int precision, const LaunchShape& ls, int mode,
                       int k_in_chunk, int parity_in, bool home_out, hipStream_t st) {
    if (!s.src2 || (precision != 0 && (!s.srcm || !s.srcm2))) return hipErrorInvalidValue;
    RowsArgs A{};
    double4* buf[2] = {s.src, s.src2};
    MixedSrc* bufm[2] = {s.srcm, s.srcm2};
    A.src_in = buf[parity_in];
    A.src_out = home_out ? buf[0] : buf[1 - parity_in];
    A.srcm_in = precision == 0 ? nullptr : bufm[parity_in];
    A.srcm_out = precision == 0 ? nullptr : (home_out ? bufm[0] : bufm[1 - parity_in]);
    A.vx = s.vx;
    A.vy = s.vy;
    A.vz = s.vz;
    A.ax = s.ax;
    A.ay = s.ay;
    A.az = s.az;
    A.qm = s.qm;
    A.qe = s.qe;
    A.mass = s.mass;
    A.species = s.species;
    A.traps = s.traps;
    A.cool = s.cool;
    A.counter = s.counter;
    A.vacc = s.vacc;
    A.vavg = s.vavg;
    A.n = s.n;
    A.n_pad = s.n_pad;
    switch (precision) {
        case 0: return rows_dispatch<0>(A, ls.rows_tr, ls.cool_on, mode, k_in_chunk, st);
        case 2: return rows_dispatch<2>(A, ls.rows_tr, ls.cool_on, mode, k_in_chunk, st);
        default: return rows_dispatch<1>(A, ls.rows_tr, ls.cool_on, mode, k_in_chunk, st);
    }
}

hipError_t launch_counter_add(const DevState& s, int64_t k, hipStream_t st) {
    k_counter_add<<<1, 64, 0, st>>>(s.counter, k);
    return hipGetLastError();
}

hipError_t launch_coulomb_potential(const DevState& s, int, hipStream_t st) {
    k_coulomb_potential<<<blocks_for(s.n, 256), 256, 0, st>>>(s.src, s.qe, s.trap_of, s.offsets,
                                                              s.n, s.scratch);
    return hipGetLastError();
}

hipError_t launch_check_finite(const DevState& s, hipStream_t st) {
    k_check_finite<<<blocks_for(s.n, 256), 256, 0, st>>>(s.src, s.vx, s.vy, s.vz, s.n, s.flags);
    return hipGetLastError();
}

hipError_t launch_count_lost(const DevState& s, double r_lost, hipStream_t st) {
    k_count_lost<<<blocks_for(s.n, 256), 256, 0, st>>>(s.src, s.n, r_lost * r_lost, s.flags + 1);
    return hipGetLastError();
}

}  // namespace lion
