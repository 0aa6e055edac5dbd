// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace lion {

// CODATA 2018 / SI 2019.
constexpr double kElementaryCharge = 1.602176634e-19;  // C
constexpr double kEps0 = 8.8541878128e-12;             // F/m
constexpr double kAmu = 1.66053906660e-27;             // kg
constexpr double kPi = 3.14159265358979323846;

// Float-float positions of the FP32 pair path are stored in units of
// 2^-20 m (~0.95 um) so that inter-ion distances are O(1) and r^-3 of close
// pairs stays far from the FP32 range limits; the power of two keeps the
// rescaling exact.
constexpr double kMixedScale = 1048576.0;             // 2^20 per metre
constexpr double kMixedFieldScale = 1099511627776.0;  // 2^40 = kMixedScale^2

// Lower bound added to r^2 so that the self pair and exactly coincident ions
// give a finite r^-3 multiplying an exactly zero difference (contribution 0).
constexpr double kR2FloorF64 = 1e-200;  // m^2
constexpr float kR2FloorF32 = 1e-20f;   // (2^-20 m)^2

// Per-trap parameters in device memory.  The rf phase uses
// t = t_start + k dt evaluated in FP64 with k the step index inside the
// current lion_step call.
struct TrapDev {
    double a_rf;     // V0 / R0^2                     (V/m^2)
    double omega;    // Omega                         (rad/s)
    double a_dc;     // kappa U0 / Z0^2               (V/m^2)
    double f;        // exp(-gamma dt / 2)
    double dt;       // s
    double h;        // dt / 2
    double t_start;  // s
    double gamma;    // 1/s (kept for reference)
    double ps;       // pseudopotential trap: A_rf^2 / (2 Omega^2); 0 for the full rf field
};

// Cooling in the velocity half-steps (applied after the isotropic damping):
// beams decay the velocity component along k by f = exp(-gamma dt/2); baths
// apply v <- c1 v + sqrt(k_B T / M (1 - c1^2)) xi with Philox4x32-10 normals.
constexpr int kMaxBeams = 4;
constexpr int kMaxBaths = 4;
constexpr double kBoltzmann = 1.380649e-23;  // J/K

struct BeamDev {
    double kx, ky, kz;  // unit direction
    double f;           // exp(-gamma dt / 2) for the current step size
    int32_t species;    // -1: every species
    int32_t on;
    int32_t pad[2];
};

struct BathDev {
    double c1;           // exp(-dt / (2 tau))
    double kt;           // k_B T
    double omc2;         // 1 - c1^2; the kernel forms sqrt(kt / M * omc2)
    uint64_t seed;
    int32_t species;     // -1: every species
    int32_t on;
};

struct CoolDev {
    BeamDev beams[kMaxBeams];
    BathDev baths[kMaxBaths];
    int32_t nbeams;      // highest active beam index + 1 (0: none)
    int32_t nbaths;
    int64_t step_base;   // steps completed before the current lion_step call
    // time average of the velocities: window length in steps (0: off) and the
    // run-wide step count at which the averaging was (re)started
    int32_t avg_window;
    int32_t avg_pad;
    int64_t avg_origin;
};

// Minimisation state in device memory: parameters, the last reduction and
// the iteration count (kernels read the parameters here, so one captured
// graph serves every call).
struct MinDev {
    double dt, dmax, ftol;
    double P, FF, fmax;   // v.F, F.F, max |F| at the current positions
    int64_t iterations;   // iterations that moved the ions
    int64_t max_iter;
    int32_t done;         // fmax <= ftol or iterations >= max_iter
    int32_t pad;
};

// Rigid body: a group of ions that keeps its shape.  Member i sits at
// R + A(q) d_i (d_i fixed in the body frame) and moves with V + w x A(q) d_i.
struct RigidDev {
    double M;         // mass (kg)
    double inv_i[3];  // inverse principal moments (0 for a vanishing moment)
    double q[4];      // orientation quaternion (w, x, y, z), body frame -> space
    double R[3];      // centre of mass
    double V[3];      // COM velocity
    double L[3];      // angular momentum about the COM (space frame)
    double F[3];      // total force on the members at the current positions
    double T[3];      // torque about the COM at the current positions
    double w[3];      // angular velocity (space frame)
    double pad;
};

// Body state built on the host from ion positions and velocities.
struct RigidHost {
    int32_t nbodies = 0;
    std::vector<RigidDev> bodies;   // [nbodies]
    std::vector<int32_t> rb;        // [n] dense body index per ion, -1 for free ions
    std::vector<int32_t> members;   // ion indices grouped by body, ascending within a body
    std::vector<int32_t> start;     // [nbodies + 1] offsets into members
    std::vector<double> dbody;      // [3][n] body-frame offsets (0 for free ions)
    std::vector<double> vx, vy, vz; // [n] velocities with members set to the rigid motion
};

// Builds the body state of the groups body[i] >= 0 (lion_rigid_host.cpp).
// Returns 0, or -1 when a body has a non-positive total mass.
int rigid_build(int64_t n, const double* mass, const double* x, const double* y,
                const double* z, const double* vx, const double* vy, const double* vz,
                const int32_t* body, RigidHost& out);

// One ion of the FP32 pair stream: high and low float parts of the scaled
// position and the negated charge in units of e.
struct MixedSrc {
    float xh, yh, zh, nq;
    float xl, yl, zl, r2floor;  // r2floor = kR2FloorF32 (read as an operand)
};

enum UpdateMode : int {
    kModeAccel = 0,      // a <- a(x, t) only
    kModeEnd = 1,        // a <- a(x, t); v <- f (v + h a)
    kModeEndDrift = 2,   // kModeEnd, then the first half of the next step
};

// Device arrays carved from the caller's workspace.
struct DevState {
    int64_t n;        // ions (all traps)
    int64_t n_pad;    // padded length of the per-ion arrays
    double4* src;     // [n_pad] {x, y, z, 1.5 q/e}: positions + FP64 source stream
    MixedSrc* srcm;   // [n_pad] FP32 source stream (mixed precisions only)
    double* vx;
    double* vy;
    double* vz;
    double* ax;
    double* ay;
    double* az;
    double* qm;       // Q / M per ion
    double* qe;       // Q / e per ion
    double* mass;     // kg
    int32_t* trap_of; // trap index per ion
    double* part;     // [j_split][3][n_pad] partial field sums
    double* scratch;  // [n_pad] per-ion diagnostics
    TrapDev* traps;   // [n_traps]
    int64_t* offsets; // [n_traps + 1]
    int32_t* order;   // [n_traps] launch order (largest trap first)
    int64_t* counter; // step index inside the current call
    int32_t* flags;   // [4] diagnostics (non-finite count)
    CoolDev* cool;    // beams, baths and the velocity time average
    int32_t* species; // [n_pad] species label per ion (default 0)
    double* vacc;     // [3][n_pad] velocity sums of the open averaging window
    double* vavg;     // [3][n_pad] average of the last completed window
    MinDev* minst;       // minimisation state
    double* minpart;     // [3 * blocks of 256 ions] partial reductions
    // rigid-body integration (NULL / 0 when off)
    int32_t nbodies;
    RigidDev* rigid;     // [nbodies]
    int32_t* rb;         // [n_pad] dense body index per ion, -1 for free ions
    double* dbody;       // [3][n_pad] body-frame offsets of the members
    int32_t* rmembers;   // [n_pad] member ions grouped by body
    int32_t* rstart;     // [nbodies + 1]
    // rigid-body exclusion (all NULL when no bodies are set)
    int32_t* body_code;  // [n_pad] body id >= 0, or -1 - i for a free ion i
    int32_t* tile_body;  // [n_pad / 256] body of every ion of a 256-ion tile, or -1 (none, or several)
    int32_t* tile_bmin;  // [n_pad / 256] smallest body id >= 0 in a tile (INT32_MAX: none)
    int32_t* tile_bmax;  // [n_pad / 256] largest body id in a tile (-1: none)
    int32_t* body_gmin;  // [n_pad / 16] smallest body id >= 0 in each group of 16 ions
    int32_t* body_gmax;  // [n_pad / 16] largest body id (-1 if none)
    // second position buffers of the one-launch step (NULL when not allocated)
    double4* src2;
    MixedSrc* srcm2;
};

struct LaunchShape {
    int i_per_lane;
    int j_split;
    int jps;          // sources per slice (multiple of 64)
    int flush_len;
    int batch_block;
    int lds_sources;  // FP32 pair kernels: 1 = sources staged in LDS, 0 = scalar loads
    int symmetric;    // 1 = each unordered pair once (tile pairs), 0 = all ordered pairs
    int sym_variant;  // pair-once kernel variant (0-based)
    int update_waves; // waves per 64 ions in the step epilogue (4, 8 or 16)
    int small_path;   // single trap stepped by the one-workgroup kernel (k_batch, one trap)
    int batch_tpt;    // batched kernel: targets per thread for traps of >= 128 ions (0: by size)
    bool cool_on;     // a beam, bath or time average is on: the kernels built with them run
    double uniform_q;  // every ion's charge in units of e when all are equal, else 0
    int sym_masked;    // pair-once kernels with the per-pair body test (bodies share tiles)
    int rows;          // one launch per step (k_rows) for the single trap
    int rows_tr;       // targets per workgroup of that launch: 2, 4 or 8
};

// Tiles of 256 ions used by the pair kernels that evaluate each pair once; the
// epilogue then adds one partial per tile.
inline int sym_tiles(int64_t n) { return (int)((n + 255) / 256); }
constexpr int kMaxSymTiles = 512;
// Pair-once kernels by default from here: 32 tiles in every precision (measured
// crossovers; FP32 pairs with FP64 run sums moved from 40 tiles to 32 once both
// kernel families stored FP32 partials: 8192 ions 31.5 against 32.9 us per step).
constexpr int64_t kSymDefaultIons = 8192;
constexpr int64_t kSymDefaultIonsMixed = 8192;

// Kernel launchers (lion_kernels.hip).  All return hipSuccess or the launch error.
hipError_t launch_drift(const DevState& s, bool cool_on, hipStream_t st);
hipError_t launch_pair(const DevState& s, int precision, const LaunchShape& ls, bool count_step,
                       hipStream_t st);
hipError_t launch_update(const DevState& s, int precision, const LaunchShape& ls, int mode,
                         bool use_counter, hipStream_t st);
hipError_t launch_pack_mixed(const DevState& s, hipStream_t st);
// Device arrays x, y, z, charge (C), mass (kg) of s.n ions into s.src, s.srcm
// (if set), s.qm, s.qe (zero charge up to s.n_pad) and T into s.traps[0].
hipError_t launch_pack_inputs(const double* x, const double* y, const double* z,
                              const double* charge, const double* mass, const DevState& s,
                              const TrapDev& T, hipStream_t st);
// Message returned by lion_last_error(NULL) (calls without a handle).
void set_handle_free_error(const std::string& msg);
hipError_t launch_batch(const DevState& s, int precision, int n_traps, int max_trap,
                        const LaunchShape& ls, int nsteps, int mode_first, hipStream_t st);
hipError_t launch_batch_accel(const DevState& s, int precision, int n_traps, int max_trap,
                              const LaunchShape& ls, hipStream_t st);
hipError_t launch_rigid_wrench(const DevState& s, bool end_kick, hipStream_t st);
hipError_t launch_rigid_drift(const DevState& s, hipStream_t st);
hipError_t launch_rigid_place(const DevState& s, int precision, hipStream_t st);
hipError_t launch_min_reduce(const DevState& s, hipStream_t st);
hipError_t launch_min_move(const DevState& s, int precision, hipStream_t st);
hipError_t launch_hessian(const DevState& s, const TrapDev& T, double* D, hipStream_t st);
// Eigenvalues (ascending, into W) and optionally eigenvectors (into A's
// columns) of the symmetric m x m matrix A (upper triangle read) with
// rocSOLVER on the rocBLAS handle h; E is m doubles of scratch and the solver
// works in scratch (scratch_bytes from eigh_scratch_bytes).  Returns 0 or -1
// with err set (lion_modes.cpp).
int eigh_handle_create(void** h, std::string& err);
void eigh_handle_destroy(void* h);
// Solver scratch for an m x m problem, asked of rocSOLVER in rocBLAS's size
// query mode (nothing runs; the pointers are device arrays of the call's sizes).
int eigh_scratch_bytes(void* h, int m, bool vectors, double* A, double* W, double* E, int* info,
                       size_t* bytes, std::string& err);
int eigh_device(void* h, double* A, int m, double* W, double* E, int* info, bool vectors,
                void* scratch, size_t scratch_bytes, hipStream_t st, std::string& err);
// One step (or, with kModeAccel, one force evaluation) of one trap in a single
// launch: positions read from buffer parity_in (0: src/srcm, 1: src2/srcm2);
// drifted positions written to the other buffer, or with home_out to buffer 0.
hipError_t launch_rows(const DevState& s, int precision, const LaunchShape& ls, int mode,
                       int k_in_chunk, int parity_in, bool home_out, hipStream_t st);
hipError_t launch_counter_add(const DevState& s, int64_t k, hipStream_t st);
hipError_t launch_coulomb_potential(const DevState& s, int n_traps, hipStream_t st);
hipError_t launch_check_finite(const DevState& s, hipStream_t st);
// Counts ions beyond r_lost (m) of the trap centre, or non-finite, into flags[1].
hipError_t launch_count_lost(const DevState& s, double r_lost, hipStream_t st);

}  // namespace lion
