// C ABI of the trapped-ion engine: argument checking, workspace carving,
// launch-shape choice and launch-graph caching around the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "lion.h"
#include "lion_internal.h"

using lion::DevState;
using lion::LaunchShape;
using lion::TrapDev;

struct lion_sim {
    int precision = 0;
    int64_t n = 0;
    int32_t n_traps = 1;
    bool batched = false;
    int max_trap = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    DevState d{};
    LaunchShape ls{};
    lion_kernel_config cfg{};
    int j_max = 1;
    std::vector<TrapDev> traps;     // host mirror
    std::vector<double> t_now;      // per-trap clock
    std::vector<int64_t> offsets;   // [n_traps + 1]
    std::vector<double> mass, charge;
    bool state_set = false;
    bool has_bodies = false;
    int64_t steps_done = 0;           // run-wide step count (numbers the bath draws)
    double uniform_q = 0.0;           // common charge (units of e) of all ions, 0 if they differ
    bool rigid_on = false;            // rigid-body integration of the body groups
    std::vector<int32_t> rigid_ids;   // [n] body id per ion while rigid_on
    size_t rigid_off[5] = {0, 0, 0, 0, 0};  // workspace offsets: bodies, rb, dbody, members, start
    int32_t avg_window = 0;           // velocity time average: window in steps (0: off)
    int64_t avg_origin = 0;           // steps_done when the averaging was (re)started
    struct Beam { double kx, ky, kz, gamma; int32_t species; };
    struct Bath { double temperature, tau; uint64_t seed; int32_t species; };
    Beam beams[lion::kMaxBeams] = {};
    Bath baths[lion::kMaxBaths] = {};
    lion::CoolDev cool{};
    char* ws = nullptr;
    size_t body_off[5] = {0, 0, 0, 0, 0};
    bool tile_bodies = false;  // every 256-ion tile holds ions of one body only, or none
    std::map<std::pair<int64_t, int>, hipGraphExec_t> graphs;  // (chunk length, kind)
    void* eigh = nullptr;  // rocBLAS handle of the normal-mode solver (created on first use)
    std::string err;
};

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxTrap = 1024;
// traps of at most this many ions step on one wave (the one-wave kernel, us per
// step FP64 / FP32 pairs / compensated against 256 threads: 16 ions 0.69 / 0.75 /
// 0.83 against 1.14 / 1.29 / 1.16; 20 ions 1.12 / 1.13 / 1.36 against 1.14 / 1.29
// / 1.16)
constexpr int64_t kOneWaveIons = 16;
// steps per captured launch when not set: 1000 where one workgroup steps a trap
// for the whole launch and a step takes a microsecond or two (a single trap of
// <= LION_SMALL_TRAP_IONS, or batches of traps of <= 64 ions; 8 ions: 0.60
// against 0.67 us per step with 100, before the one-wave kernel's unrolled
// butterfly), else 100
constexpr int kChunkLong = 1000;
constexpr int kChunkDefault = 100;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int64_t padded(int64_t n) { return round_up(std::max<int64_t>(n, 1), 1024); }

// Upper bound on source slices for n ions: at most 64, at most one slice per 64
// sources, and partial sums kept under ~400 MB for very large n.
int j_max_for(int64_t n) {
    int64_t j = std::min<int64_t>(64, std::max<int64_t>(1, (int64_t(1) << 24) / std::max<int64_t>(n, 1)));
    j = std::min<int64_t>(j, std::max<int64_t>(1, round_up(n, 64) / 64));
    return (int)j;
}

// Partial-sum slices the workspace holds: enough for any source split and, up
// to kMaxSymTiles tiles, for the pair-once kernels (one slice per tile; at
// N = 131072 that is 512 slices, 1.6 GB).
int slices_for(int64_t n) {
    const int nb = lion::sym_tiles(n);
    return std::max(j_max_for(n), nb <= lion::kMaxSymTiles ? nb : 0);
}

struct Layout {
    size_t src, srcm, v, a, qm, qe, mass, trap_of, part, scratch, traps, offsets, order, counter,
        flags, body_code, tile_body, tile_brange, body_gmin, body_gmax, cool, species, vacc, vavg, rigid, rb, dbody,
        rmembers, rstart, minst, minpart, src2, srcm2, total;
};

Layout layout_for(int64_t n, int32_t n_traps, int precision, bool batched) {
    const int64_t np = padded(n);
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.src = take(np * sizeof(double4));
    L.srcm = (precision != LION_FP64 && !batched) ? take(np * sizeof(lion::MixedSrc)) : SIZE_MAX;
    L.v = take(3 * np * sizeof(double));
    L.a = take(3 * np * sizeof(double));
    L.qm = take(np * sizeof(double));
    L.qe = take(np * sizeof(double));
    L.mass = take(np * sizeof(double));
    L.trap_of = take(np * sizeof(int32_t));
    L.part = batched ? SIZE_MAX : take((size_t)slices_for(n) * 3 * np * sizeof(double));
    L.scratch = take(np * sizeof(double));
    L.traps = take((size_t)n_traps * sizeof(TrapDev));
    L.offsets = take((size_t)(n_traps + 1) * sizeof(int64_t));
    L.order = take((size_t)n_traps * sizeof(int32_t));
    L.counter = take(sizeof(int64_t));
    L.flags = take(4 * sizeof(int32_t));
    L.body_code = take(np * sizeof(int32_t));
    L.tile_body = take(np / 256 * sizeof(int32_t));
    L.tile_brange = take(2 * (np / 256) * sizeof(int32_t));
    L.body_gmin = take(np / 16 * sizeof(int32_t));
    L.body_gmax = take(np / 16 * sizeof(int32_t));
    L.cool = take(sizeof(lion::CoolDev));
    L.species = take(np * sizeof(int32_t));
    L.vacc = take(3 * np * sizeof(double));
    L.vavg = take(3 * np * sizeof(double));
    // rigid bodies (single trap only): room for one body per ion
    L.rigid = batched ? SIZE_MAX : take(np * sizeof(lion::RigidDev));
    L.rb = batched ? SIZE_MAX : take(np * sizeof(int32_t));
    L.dbody = batched ? SIZE_MAX : take(3 * np * sizeof(double));
    L.rmembers = batched ? SIZE_MAX : take(np * sizeof(int32_t));
    L.rstart = batched ? SIZE_MAX : take((np + 1) * sizeof(int32_t));
    L.minst = take(sizeof(lion::MinDev));
    L.minpart = take((size_t)3 * ((np + 255) / 256) * sizeof(double));
    // second position buffers of the one-launch step (single trap)
    L.src2 = batched ? SIZE_MAX : take(np * sizeof(double4));
    L.srcm2 = (precision != LION_FP64 && !batched) ? take(np * sizeof(lion::MixedSrc)) : SIZE_MAX;
    L.total = o;
    return L;
}

bool is_fin(double v) { return std::isfinite(v); }

int fail(lion_sim* s, int code, const std::string& msg) {
    if (s) s->err = msg;
    return code;
}

int hip_fail(lion_sim* s, hipError_t e, const char* where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(s, LION_ERR_HIP, m);
}

#define LION_HIP(s, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail((s), e_, #call); \
    } while (0)

void default_shape(lion_sim* s) {
    LaunchShape& ls = s->ls;
    const int64_t n = s->n;
    const bool mixed = s->precision != LION_FP64;
    // all-pairs shapes: one target per lane and many source slices below 16384
    // ions (measured best up to 10000), several targets per lane above
    ls.i_per_lane = s->cfg.i_per_lane > 0 ? s->cfg.i_per_lane
                                          : (n >= 16384 ? (mixed ? 4 : 2) : 1);
    ls.flush_len = s->cfg.flush_len > 0 ? s->cfg.flush_len : 8;
    ls.batch_block = s->cfg.batch_block > 0 ? s->cfg.batch_block : 256;
    ls.lds_sources = s->cfg.lds_sources > 0 ? (s->cfg.lds_sources == 2 ? 1 : 0) : 1;
    const int nb = lion::sym_tiles(n);
    // pair-once kernels: when asked for, and by default for one trap from the
    // size where they measured faster (8192 ions; from 12288 on by a wide margin
    // in every precision)
    const bool sym_ok = nb <= lion::kMaxSymTiles && !s->batched;
    const int64_t sym_from = s->precision == LION_MIXED_F64ACC ? lion::kSymDefaultIonsMixed
                                                                : lion::kSymDefaultIons;
    const bool sym_default = s->cfg.symmetric <= 0 && n >= sym_from;
    ls.symmetric = (sym_ok && (s->cfg.symmetric == 2 || sym_default)) ? 1 : 0;
    // bodies that share tiles with other ions need the per-pair test in those kernels
    ls.sym_masked = (ls.symmetric && s->has_bodies && !s->tile_bodies) ? 1 : 0;
    // built-in pair-once variant: the fastest measured (9 for FP32 pairs: 72.6 against
    // 74.9 us for 7 at 16384 ions, 997 against 1029 us at 65536; 6 for FP64)
    ls.sym_variant = s->cfg.sym_variant > 0 ? s->cfg.sym_variant - 1 : (mixed ? 8 : 5);
    const int64_t n64 = round_up(n, 64);
    const int64_t blocks_x = (n + 64 * ls.i_per_lane - 1) / (64 * ls.i_per_lane);
    int j;
    if (s->cfg.j_split > 0) {
        j = s->cfg.j_split;
    } else {
        // aim for ~1024 blocks of 4 waves (4 waves per SIMD on 256 CUs), ~4096
        // below 16384 ions, where more, shorter slices measured faster
        const int64_t target = n >= 16384 ? 1024 : 4096;
        j = (int)std::max<int64_t>(1, (target + blocks_x - 1) / blocks_x);
    }
    j = std::max(1, std::min(j, s->j_max));
    ls.jps = (int)round_up((n64 + j - 1) / j, 64);
    ls.j_split = (int)((n64 + ls.jps - 1) / ls.jps);  // slices that hold sources
    if (ls.symmetric) ls.j_split = nb;               // one partial per tile
    // epilogue: 4 waves per 64 ions unless set (8 and 16 measured no faster)
    ls.update_waves = s->cfg.update_waves > 0 ? s->cfg.update_waves : 4;
    // one launch per step: asked for, or built in up to LION_ONE_LAUNCH_IONS on the
    // all-pairs kernels (FP64, us per step against the pair kernel + epilogue: 200
    // ions 3.7 / 6.0, 1024 ions 4.9 / 6.3, 2048 ions 7.3 / 8.2); one target per
    // workgroup up to 1024 ions, two above (2048 ions: 8.7 against 7.3 us)
    ls.rows = (!s->batched && (s->cfg.step_launches == 1 ||
                               (s->cfg.step_launches <= 0 && !ls.symmetric &&
                                n <= LION_ONE_LAUNCH_IONS)))
                  ? 1
                  : 0;
    ls.rows_tr = n <= 1024 ? 1 : 2;
    ls.uniform_q = s->uniform_q;
    ls.batch_tpt = s->cfg.batch_tpt > 0 ? s->cfg.batch_tpt : 0;
    ls.small_path = s->cfg.small_trap > 0 ? (s->cfg.small_trap == 2 ? 1 : 0)
                                          : (n <= LION_SMALL_TRAP_IONS ? 1 : 0);
    // one-workgroup stepping of a single trap: 256 threads up to 32 ions, 512 up
    // to 64, then 1024 (measured per size; e.g. 64 ions: 1.94 us per step at 512
    // against 2.13 at 256 and 2.27 at 1024)
    if (!s->batched && ls.small_path && s->cfg.batch_block <= 0)
        ls.batch_block = n <= kOneWaveIons ? 64 : (n <= 32 ? 256 : (n <= 64 ? 512 : 1024));
    // batches whose largest trap holds 256 ions or more: 1024 threads per trap
    // (the 512-trap batch of 2-512 ions: 4.0 against 6.8 ms per 100 steps at 256)
    if (s->batched && s->cfg.batch_block <= 0 && s->max_trap >= 256) ls.batch_block = 1024;
    if (s->batched && s->cfg.batch_block <= 0 && s->max_trap <= kOneWaveIons) ls.batch_block = 64;
}

void clear_graphs(lion_sim* s) {
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    s->graphs.clear();
}

int upload_traps(lion_sim* s) {
    LION_HIP(s, hipMemcpyAsync(s->d.traps, s->traps.data(), s->traps.size() * sizeof(TrapDev),
                               hipMemcpyHostToDevice, s->stream));
    return LION_OK;
}

// Half-step factors of the beams and baths for step size dt, and the run-wide
// step count, into device memory.  Uses one dt for every trap (the first).
int upload_cooling(lion_sim* s, double dt) {
    const double h = 0.5 * dt;
    lion::CoolDev& C = s->cool;
    C.nbeams = C.nbaths = 0;
    for (int b = 0; b < lion::kMaxBeams; ++b) {
        const auto& B = s->beams[b];
        lion::BeamDev& D = C.beams[b];
        D.on = B.gamma > 0.0;
        D.kx = B.kx;
        D.ky = B.ky;
        D.kz = B.kz;
        D.f = std::exp(-(B.gamma * h));
        D.species = B.species;
        if (D.on) C.nbeams = b + 1;
    }
    for (int c = 0; c < lion::kMaxBaths; ++c) {
        const auto& T = s->baths[c];
        lion::BathDev& D = C.baths[c];
        D.on = T.tau > 0.0;
        D.c1 = D.on ? std::exp(-(h / T.tau)) : 1.0;
        D.kt = lion::kBoltzmann * T.temperature;
        D.omc2 = 1.0 - D.c1 * D.c1;
        D.seed = T.seed;
        D.species = T.species;
        if (D.on) C.nbaths = c + 1;
    }
    C.step_base = s->steps_done;
    C.avg_window = s->avg_window;
    C.avg_origin = s->avg_origin;
    // captured graphs hold the kernels built with or without these features
    const bool on = C.nbeams > 0 || C.nbaths > 0 || C.avg_window > 0;
    if (on != s->ls.cool_on) {
        LION_HIP(s, hipStreamSynchronize(s->stream));  // no launch of a graph still pending
        clear_graphs(s);
        s->ls.cool_on = on;
    }
    LION_HIP(s, hipMemcpyAsync(s->d.cool, &s->cool, sizeof(lion::CoolDev), hipMemcpyHostToDevice,
                               s->stream));
    return LION_OK;
}

// A single trap stepped inside one workgroup (the batched kernel with one trap).
bool small_path_active(const lion_sim* s) {
    return !s->batched && s->ls.small_path && s->n <= kMaxTrap && !s->has_bodies &&
           s->d.nbodies == 0;
}

// The single trap steps with one launch per step (k_rows).
bool rows_active(const lion_sim* s) {
    return !s->batched && s->ls.rows && !small_path_active(s) && !s->has_bodies &&
           s->d.nbodies == 0 && s->d.src2 && (s->precision == LION_FP64 || s->d.srcm2);
}

// Steps per captured launch: the configured count, else the built-in one.
int64_t chunk_len(const lion_sim* s) {
    if (s->cfg.chunk_steps > 0) return s->cfg.chunk_steps;
    const bool one_wg = small_path_active(s) || (s->batched && s->max_trap <= 64);
    return one_wg ? kChunkLong : kChunkDefault;
}

// Accelerations at the current positions and clocks, by the kernels that step
// the handle (so a trap stepped inside one workgroup gets them from that kernel).
int refresh_accel(lion_sim* s) {
    for (int k = 0; k < s->n_traps; ++k) s->traps[k].t_start = s->t_now[k];
    int rc = upload_traps(s);
    if (rc) return rc;
    if (s->batched || small_path_active(s)) {
        LION_HIP(s, hipMemsetAsync(s->d.counter, 0, sizeof(int64_t), s->stream));
        LION_HIP(s, lion::launch_batch_accel(s->d, s->precision, s->n_traps, s->max_trap, s->ls,
                                             s->stream));
        return LION_OK;
    }
    if (rows_active(s)) {
        LION_HIP(s, lion::launch_rows(s->d, s->precision, s->ls, lion::kModeAccel, 0, 0, true,
                                      s->stream));
        return LION_OK;
    }
    LION_HIP(s, lion::launch_pair(s->d, s->precision, s->ls, false, s->stream));
    LION_HIP(s, lion::launch_update(s->d, s->precision, s->ls, lion::kModeAccel, false, s->stream));
    return LION_OK;
}

// Kernels of one chunk of L steps on stream st.
hipError_t enqueue_chunk(lion_sim* s, int64_t L, hipStream_t st) {
    hipError_t e;
    if (s->batched) {
        e = lion::launch_batch(s->d, s->precision, s->n_traps, s->max_trap, s->ls, (int)L, 0, st);
        if (e != hipSuccess) return e;
        return lion::launch_counter_add(s->d, L, st);
    }
    if (small_path_active(s)) {
        // the whole trap inside one workgroup, L steps per launch
        e = lion::launch_batch(s->d, s->precision, 1, (int)s->n, s->ls, (int)L, 0, st);
        if (e == hipSuccess) e = lion::launch_counter_add(s->d, L, st);
        if (e == hipSuccess && s->d.srcm) e = lion::launch_pack_mixed(s->d, st);
        return e;
    }
    const bool rigid = s->d.nbodies > 0;
    if (rows_active(s)) {
        // one launch per step; positions alternate between the two buffers and
        // the last step of the chunk leaves them in the first
        e = lion::launch_drift(s->d, s->ls.cool_on, st);
        for (int64_t k = 0; k < L && e == hipSuccess; ++k) {
            const bool last = k + 1 == L;
            e = lion::launch_rows(s->d, s->precision, s->ls,
                                  last ? lion::kModeEnd : lion::kModeEndDrift, (int)k,
                                  (int)(k & 1), last, st);
        }
        if (e == hipSuccess) e = lion::launch_counter_add(s->d, L, st);
        return e;
    }
    if (rigid) {
        // force and torque at the starting positions, then the bodies' first half-step
        e = lion::launch_rigid_wrench(s->d, false, st);
        if (e != hipSuccess) return e;
    }
    e = lion::launch_drift(s->d, s->ls.cool_on, st);
    if (e != hipSuccess) return e;
    if (rigid) {
        e = lion::launch_rigid_drift(s->d, st);
        if (e == hipSuccess) e = lion::launch_rigid_place(s->d, s->precision, st);
        if (e != hipSuccess) return e;
    }
    for (int64_t k = 0; k < L; ++k) {
        e = lion::launch_pair(s->d, s->precision, s->ls, true, st);
        if (e != hipSuccess) return e;
        const int mode = (k + 1 < L) ? lion::kModeEndDrift : lion::kModeEnd;
        e = lion::launch_update(s->d, s->precision, s->ls, mode, true, st);
        if (e != hipSuccess) return e;
        if (rigid) {
            e = lion::launch_rigid_wrench(s->d, true, st);
            if (e == hipSuccess && k + 1 < L) {
                e = lion::launch_rigid_drift(s->d, st);
                if (e == hipSuccess) e = lion::launch_rigid_place(s->d, s->precision, st);
            }
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// The captured graph of a chunk of L steps, captured and instantiated on
// first use.
int chunk_graph(lion_sim* s, int64_t L, hipGraphExec_t* out) {
    auto key = std::make_pair(L, 0);
    auto it = s->graphs.find(key);
    if (it == s->graphs.end()) {
        hipGraph_t g = nullptr;
        LION_HIP(s, hipStreamBeginCapture(s->capture, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_chunk(s, L, s->capture);
        hipError_t e2 = hipStreamEndCapture(s->capture, &g);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(s, e, "capture chunk");
        }
        if (e2 != hipSuccess) return hip_fail(s, e2, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(s, e, "hipGraphInstantiate");
        it = s->graphs.emplace(key, ex).first;
        // resident on the device now rather than at the first launch
        LION_HIP(s, hipGraphUpload(ex, s->stream));
    }
    *out = it->second;
    return LION_OK;
}

int run_chunk(lion_sim* s, int64_t L) {
    if (s->cfg.use_graph == 2) {
        LION_HIP(s, enqueue_chunk(s, L, s->stream));
        return LION_OK;
    }
    hipGraphExec_t ex = nullptr;
    int rc = chunk_graph(s, L, &ex);
    if (rc) return rc;
    LION_HIP(s, hipGraphLaunch(ex, s->stream));
    return LION_OK;
}

// Whether the cooling kernels are needed by the current beams, baths and time
// average (the launch graphs hold kernels built with or without them).
bool cooling_on(const lion_sim* s) {
    bool on = s->avg_window > 0;
    for (const auto& B : s->beams) on = on || B.gamma > 0.0;
    for (const auto& T : s->baths) on = on || T.tau > 0.0;
    return on;
}

// K minimisation iterations: reduce + stopping test, move, forces at the new
// positions (a graph per K, parameters read from device memory).
hipError_t enqueue_min_chunk(lion_sim* s, int64_t K, hipStream_t st) {
    for (int64_t k = 0; k < K; ++k) {
        hipError_t e = lion::launch_min_reduce(s->d, st);
        if (e == hipSuccess) e = lion::launch_min_move(s->d, s->precision, st);
        if (e == hipSuccess) e = lion::launch_pair(s->d, s->precision, s->ls, false, st);
        if (e == hipSuccess)
            e = lion::launch_update(s->d, s->precision, s->ls, lion::kModeAccel, false, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int run_min_chunk(lion_sim* s, int64_t K) {
    if (s->cfg.use_graph == 2) {
        LION_HIP(s, enqueue_min_chunk(s, K, s->stream));
        return LION_OK;
    }
    auto key = std::make_pair(K, 1);
    auto it = s->graphs.find(key);
    if (it == s->graphs.end()) {
        hipGraph_t g = nullptr;
        LION_HIP(s, hipStreamBeginCapture(s->capture, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_min_chunk(s, K, s->capture);
        hipError_t e2 = hipStreamEndCapture(s->capture, &g);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(s, e, "capture minimisation chunk");
        }
        if (e2 != hipSuccess) return hip_fail(s, e2, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(s, e, "hipGraphInstantiate");
        it = s->graphs.emplace(key, ex).first;
    }
    LION_HIP(s, hipGraphLaunch(it->second, s->stream));
    return LION_OK;
}

int check_ws(lion_sim* s, void* ws, size_t bytes, size_t need) {
    if (!ws) return fail(s, LION_ERR_WORKSPACE, "workspace pointer is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(s, LION_ERR_WORKSPACE, "workspace not 256-byte aligned");
    if (bytes < need)
        return fail(s, LION_ERR_WORKSPACE,
                    "workspace too small: need " + std::to_string(need) + " bytes, got " +
                        std::to_string(bytes));
    return LION_OK;
}

// Message of the last failed call without a handle on this thread (a failed
// create, the allocation-free force evaluation).
thread_local std::string g_create_err;

int create_common(lion_sim** out, int32_t n_traps, const int64_t* n_per_trap, int64_t n,
                  const double* masses, const double* charges, int precision, void* ws,
                  size_t ws_bytes, void* stream, bool batched) {
    if (!out) return LION_ERR_ARG;
    *out = nullptr;
    auto* s = new lion_sim();
    auto bail = [&](int code) {
        g_create_err = s->err;
        delete s;
        return code;
    };
    if (precision < LION_FP64 || precision > LION_MIXED_KAHAN)
        return bail(fail(s, LION_ERR_ARG, "unknown precision"));
    if (n < 1) return bail(fail(s, LION_ERR_ARG, "need at least one ion"));
    if (n > (int64_t(1) << 30)) return bail(fail(s, LION_ERR_ARG, "too many ions"));
    if (!masses || !charges) return bail(fail(s, LION_ERR_ARG, "masses or charges is NULL"));
    for (int64_t i = 0; i < n; ++i) {
        if (!is_fin(masses[i]) || masses[i] <= 0.0)
            return bail(fail(s, LION_ERR_ARG, "mass " + std::to_string(i) + " not finite and > 0"));
        if (!is_fin(charges[i]))
            return bail(fail(s, LION_ERR_ARG, "charge " + std::to_string(i) + " not finite"));
    }
    s->precision = precision;
    s->n = n;
    s->n_traps = n_traps;
    s->batched = batched;
    s->stream = (hipStream_t)stream;
    s->offsets.assign(n_traps + 1, 0);
    for (int k = 0; k < n_traps; ++k) s->offsets[k + 1] = s->offsets[k] + n_per_trap[k];
    s->max_trap = 0;
    for (int k = 0; k < n_traps; ++k) s->max_trap = std::max<int>(s->max_trap, (int)n_per_trap[k]);
    Layout L = layout_for(n, n_traps, precision, batched);
    int rc = check_ws(s, ws, ws_bytes, L.total);
    if (rc) return bail(rc);
    if (hipGetDevice(&s->device) != hipSuccess) return bail(fail(s, LION_ERR_HIP, "hipGetDevice failed"));
    if (hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(s, LION_ERR_HIP, "hipStreamCreateWithFlags failed"));
    char* base = (char*)ws;
    DevState& d = s->d;
    d.n = n;
    d.n_pad = padded(n);
    d.src = (double4*)(base + L.src);
    d.srcm = L.srcm == SIZE_MAX ? nullptr : (lion::MixedSrc*)(base + L.srcm);
    d.vx = (double*)(base + L.v);
    d.vy = d.vx + d.n_pad;
    d.vz = d.vy + d.n_pad;
    d.ax = (double*)(base + L.a);
    d.ay = d.ax + d.n_pad;
    d.az = d.ay + d.n_pad;
    d.qm = (double*)(base + L.qm);
    d.qe = (double*)(base + L.qe);
    d.mass = (double*)(base + L.mass);
    d.trap_of = (int32_t*)(base + L.trap_of);
    d.part = L.part == SIZE_MAX ? nullptr : (double*)(base + L.part);
    d.scratch = (double*)(base + L.scratch);
    d.traps = (TrapDev*)(base + L.traps);
    d.offsets = (int64_t*)(base + L.offsets);
    d.order = (int32_t*)(base + L.order);
    d.counter = (int64_t*)(base + L.counter);
    d.flags = (int32_t*)(base + L.flags);
    d.cool = (lion::CoolDev*)(base + L.cool);
    d.species = (int32_t*)(base + L.species);
    d.vacc = (double*)(base + L.vacc);
    d.vavg = (double*)(base + L.vavg);
    d.minst = (lion::MinDev*)(base + L.minst);
    d.minpart = (double*)(base + L.minpart);
    d.src2 = L.src2 == SIZE_MAX ? nullptr : (double4*)(base + L.src2);
    d.srcm2 = L.srcm2 == SIZE_MAX ? nullptr : (lion::MixedSrc*)(base + L.srcm2);
    d.nbodies = 0;  // set by lion_set_rigid_bodies
    d.rigid = nullptr;
    d.rb = nullptr;
    d.dbody = nullptr;
    d.rmembers = nullptr;
    d.rstart = nullptr;
    s->rigid_off[0] = L.rigid;
    s->rigid_off[1] = L.rb;
    s->rigid_off[2] = L.dbody;
    s->rigid_off[3] = L.rmembers;
    s->rigid_off[4] = L.rstart;
    d.body_code = nullptr;  // set by lion_set_bodies
    d.tile_body = nullptr;
    d.tile_bmin = nullptr;
    d.tile_bmax = nullptr;
    d.body_gmin = nullptr;
    d.body_gmax = nullptr;
    s->body_off[0] = L.body_code;
    s->body_off[1] = L.body_gmin;
    s->body_off[2] = L.body_gmax;
    s->body_off[3] = L.tile_body;
    s->body_off[4] = L.tile_brange;
    s->ws = base;
    s->j_max = batched ? 1 : j_max_for(n);
    s->cfg.chunk_steps = 0;
    s->cfg.use_graph = 1;
    default_shape(s);

    // per-ion constants
    const int64_t np = d.n_pad;
    std::vector<double> qm(np, 0.0), qe(np, 0.0), mass(np, 0.0);
    std::vector<int32_t> trap_of(np, 0);
    for (int k = 0; k < n_traps; ++k)
        for (int64_t i = s->offsets[k]; i < s->offsets[k + 1]; ++i) trap_of[i] = k;
    for (int64_t i = 0; i < n; ++i) {
        qm[i] = charges[i] / masses[i];
        qe[i] = charges[i] / lion::kElementaryCharge;
        mass[i] = masses[i];
    }
    s->mass.assign(masses, masses + n);
    s->charge.assign(charges, charges + n);
    {
        bool same = true;
        for (int64_t i = 1; i < n && same; ++i) same = qe[i] == qe[0];
        s->uniform_q = same ? qe[0] : 0.0;
        s->ls.uniform_q = s->uniform_q;
    }
    s->traps.assign(n_traps, TrapDev{0, 1.0, 0, 1.0, 0, 0, 0, 0});
    s->t_now.assign(n_traps, 0.0);
    std::vector<int32_t> order(n_traps);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return n_per_trap[a] > n_per_trap[b]; });
    std::vector<double4> zero_src(np, make_double4(0, 0, 0, 0));
    for (int64_t i = 0; i < n; ++i) zero_src[i].w = 1.5 * qe[i];
    hipStream_t st = s->stream;
    bool ok = hipMemcpyAsync(d.qm, qm.data(), np * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(d.qe, qe.data(), np * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(d.mass, mass.data(), np * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(d.trap_of, trap_of.data(), np * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(d.offsets, s->offsets.data(), (n_traps + 1) * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(d.order, order.data(), n_traps * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(d.src, zero_src.data(), np * sizeof(double4), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemsetAsync(d.vx, 0, 3 * np * 8, st) == hipSuccess &&
              hipMemsetAsync(d.ax, 0, 3 * np * 8, st) == hipSuccess &&
              hipMemsetAsync(d.counter, 0, 8, st) == hipSuccess &&
              hipMemsetAsync(d.flags, 0, 16, st) == hipSuccess &&
              hipMemsetAsync(d.species, 0, np * 4, st) == hipSuccess &&
              hipMemsetAsync(d.vacc, 0, 3 * np * 8, st) == hipSuccess &&
              hipMemsetAsync(d.vavg, 0, 3 * np * 8, st) == hipSuccess &&
              hipMemcpyAsync(d.cool, &s->cool, sizeof(lion::CoolDev), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(d.traps, s->traps.data(), n_traps * sizeof(TrapDev), hipMemcpyHostToDevice, st) == hipSuccess;
    if (ok && d.srcm) ok = lion::launch_pack_mixed(d, st) == hipSuccess;
    if (ok) ok = hipStreamSynchronize(st) == hipSuccess;
    if (!ok) {
        (void)hipStreamDestroy(s->capture);
        return bail(fail(s, LION_ERR_HIP, "device initialisation failed"));
    }
    g_create_err.clear();
    *out = s;
    return LION_OK;
}

int check_handle(const lion_sim* s) { return s ? LION_OK : LION_ERR_ARG; }

void rigid_off(lion_sim* s) {
    s->rigid_on = false;
    s->rigid_ids.clear();
    s->d.nbodies = 0;
    s->d.rigid = nullptr;
    s->d.rb = nullptr;
    s->d.dbody = nullptr;
    s->d.rmembers = nullptr;
    s->d.rstart = nullptr;
}

// Body state from the current device state (positions and velocities), into
// the workspace; member velocities become the rigid motion.
int rigid_setup(lion_sim* s) {
    const int64_t n = s->n, np = s->d.n_pad;
    hipStream_t st = s->stream;
    std::vector<double4> src(n);
    std::vector<double> x(n), y(n), z(n), vx(n), vy(n), vz(n);
    LION_HIP(s, hipMemcpyAsync(src.data(), s->d.src, n * sizeof(double4), hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipMemcpyAsync(vx.data(), s->d.vx, n * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipMemcpyAsync(vy.data(), s->d.vy, n * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipMemcpyAsync(vz.data(), s->d.vz, n * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i) {
        x[i] = src[i].x;
        y[i] = src[i].y;
        z[i] = src[i].z;
    }
    lion::RigidHost h;
    if (lion::rigid_build(n, s->mass.data(), x.data(), y.data(), z.data(), vx.data(), vy.data(),
                          vz.data(), s->rigid_ids.data(), h) != 0)
        return fail(s, LION_ERR_ARG, "a rigid body has no mass");
    char* base = s->ws;
    auto* bodies = (lion::RigidDev*)(base + s->rigid_off[0]);
    auto* rb = (int32_t*)(base + s->rigid_off[1]);
    auto* dbody = (double*)(base + s->rigid_off[2]);
    auto* members = (int32_t*)(base + s->rigid_off[3]);
    auto* start = (int32_t*)(base + s->rigid_off[4]);
    std::vector<int32_t> rbp(np, -1);
    std::copy(h.rb.begin(), h.rb.end(), rbp.begin());
    std::vector<double> db(3 * np, 0.0);
    for (int c = 0; c < 3; ++c)
        std::copy(h.dbody.begin() + c * n, h.dbody.begin() + (c + 1) * n, db.begin() + c * np);
    if (h.nbodies > 0) {
        LION_HIP(s, hipMemcpyAsync(bodies, h.bodies.data(), h.nbodies * sizeof(lion::RigidDev),
                                   hipMemcpyHostToDevice, st));
        LION_HIP(s, hipMemcpyAsync(members, h.members.data(), h.members.size() * 4,
                                   hipMemcpyHostToDevice, st));
    }
    LION_HIP(s, hipMemcpyAsync(rb, rbp.data(), np * 4, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipMemcpyAsync(dbody, db.data(), 3 * np * 8, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipMemcpyAsync(start, h.start.data(), h.start.size() * 4, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipMemcpyAsync(s->d.vx, h.vx.data(), n * 8, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipMemcpyAsync(s->d.vy, h.vy.data(), n * 8, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipMemcpyAsync(s->d.vz, h.vz.data(), n * 8, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipStreamSynchronize(st));
    s->d.nbodies = h.nbodies;
    s->d.rigid = bodies;
    s->d.rb = rb;
    s->d.dbody = dbody;
    s->d.rmembers = members;
    s->d.rstart = start;
    return LION_OK;
}

}  // namespace

void lion::set_handle_free_error(const std::string& msg) { g_create_err = msg; }

namespace {

// Bytes of the fixed part of the normal-mode workspace: the (3n)^2 matrix, two
// vectors of 3n and the solver's status word.
size_t modes_fixed_bytes(int64_t n) {
    const size_t m = (size_t)(3 * n);
    return align_up(m * m * 8) + 2 * align_up(m * 8) + align_up(sizeof(int));
}

int modes_handle(lion_sim* s) {
    if (s->eigh) return LION_OK;
    std::string err;
    if (lion::eigh_handle_create(&s->eigh, err) != 0) return fail(s, LION_ERR_HIP, err);
    return LION_OK;
}

}  // namespace

extern "C" {

size_t lion_workspace_bytes(int64_t n_total, int32_t n_traps, int precision) {
    if (n_total < 1 || n_traps < 1 || precision < 0 || precision > 2) return 0;
    return layout_for(n_total, n_traps, precision, n_traps > 1).total;
}

int lion_create(lion_sim** out, int64_t n, const double* masses_kg, const double* charges_C,
                int precision, void* dev_workspace, size_t ws_bytes, void* hip_stream) {
    const int64_t per[1] = {n};
    return create_common(out, 1, per, n, masses_kg, charges_C, precision, dev_workspace,
                         ws_bytes, hip_stream, false);
}

int lion_create_batch(lion_sim** out, int32_t n_traps, const int64_t* n_per_trap,
                      const double* masses_kg, const double* charges_C, int precision,
                      void* dev_workspace, size_t ws_bytes, void* hip_stream) {
    if (!out) return LION_ERR_ARG;
    *out = nullptr;
    if (n_traps < 1 || !n_per_trap) {
        g_create_err = "need n_traps >= 1 and n_per_trap";
        return LION_ERR_ARG;
    }
    int64_t n = 0;
    for (int k = 0; k < n_traps; ++k) {
        if (n_per_trap[k] < 1 || n_per_trap[k] > kMaxTrap) {
            g_create_err = "trap " + std::to_string(k) + " must hold 1..1024 ions";
            return LION_ERR_ARG;
        }
        n += n_per_trap[k];
    }
    // a batch of one trap still uses the batched (workgroup-per-trap) path
    return create_common(out, n_traps, n_per_trap, n, masses_kg, charges_C, precision,
                         dev_workspace, ws_bytes, hip_stream, true);
}

int lion_set_state(lion_sim* s, const double* x, const double* y, const double* z,
                   const double* vx, const double* vy, const double* vz, double t) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (!x || !y || !z || !vx || !vy || !vz) return fail(s, LION_ERR_ARG, "state array is NULL");
    if (!is_fin(t)) return fail(s, LION_ERR_ARG, "t not finite");
    const int64_t n = s->n, np = s->d.n_pad;
    std::vector<double4> src(np, make_double4(0, 0, 0, 0));
    for (int64_t i = 0; i < n; ++i) {
        if (!is_fin(x[i]) || !is_fin(y[i]) || !is_fin(z[i]) || !is_fin(vx[i]) || !is_fin(vy[i]) ||
            !is_fin(vz[i]))
            return fail(s, LION_ERR_ARG, "state of ion " + std::to_string(i) + " not finite");
        src[i] = make_double4(x[i], y[i], z[i], 1.5 * (s->charge[i] / lion::kElementaryCharge));
    }
    LION_HIP(s, hipSetDevice(s->device));
    hipStream_t st = s->stream;
    LION_HIP(s, hipMemcpyAsync(s->d.src, src.data(), np * sizeof(double4), hipMemcpyHostToDevice, st));
    LION_HIP(s, hipMemcpyAsync(s->d.vx, vx, n * 8, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipMemcpyAsync(s->d.vy, vy, n * 8, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipMemcpyAsync(s->d.vz, vz, n * 8, hipMemcpyHostToDevice, st));
    if (s->d.srcm) LION_HIP(s, lion::launch_pack_mixed(s->d, st));
    std::fill(s->t_now.begin(), s->t_now.end(), t);
    int rc = refresh_accel(s);
    if (rc) return rc;
    LION_HIP(s, hipStreamSynchronize(st));
    s->state_set = true;
    if (s->rigid_on) return rigid_setup(s);
    return LION_OK;
}

int lion_set_trap(lion_sim* s, int32_t trap, double V_rf, double Omega, double U_dc, double r0,
                  double z0, double kappa) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (trap < -1 || trap >= s->n_traps) return fail(s, LION_ERR_ARG, "trap index out of range");
    if (!is_fin(V_rf) || !is_fin(Omega) || !is_fin(U_dc) || !is_fin(r0) || !is_fin(z0) ||
        !is_fin(kappa))
        return fail(s, LION_ERR_ARG, "trap parameter not finite");
    if (r0 <= 0 || z0 <= 0) return fail(s, LION_ERR_ARG, "r0 and z0 must be > 0");
    if (V_rf != 0.0 && Omega <= 0.0) return fail(s, LION_ERR_ARG, "Omega must be > 0 when V_rf != 0");
    const int lo = trap < 0 ? 0 : trap, hi = trap < 0 ? s->n_traps : trap + 1;
    for (int k = lo; k < hi; ++k) {
        s->traps[k].a_rf = V_rf / (r0 * r0);
        s->traps[k].omega = Omega;
        s->traps[k].a_dc = kappa * U_dc / (z0 * z0);
        s->traps[k].ps = 0.0;
    }
    LION_HIP(s, hipSetDevice(s->device));
    int rc = upload_traps(s);
    if (rc) return rc;
    if (s->state_set) return refresh_accel(s);
    return LION_OK;
}

int lion_set_pseudo_trap(lion_sim* s, int32_t trap, double V_rf, double Omega, double U_dc,
                         double r0, double z0, double kappa) {
    int rc = lion_set_trap(s, trap, V_rf, Omega, U_dc, r0, z0, kappa);
    if (rc) return rc;
    const int lo = trap < 0 ? 0 : trap, hi = trap < 0 ? s->n_traps : trap + 1;
    for (int k = lo; k < hi; ++k) {
        const double a_rf = s->traps[k].a_rf;
        s->traps[k].ps = a_rf != 0.0 ? (a_rf * a_rf) / (2.0 * Omega * Omega) : 0.0;
    }
    rc = upload_traps(s);
    if (rc) return rc;
    if (s->state_set) return refresh_accel(s);
    return LION_OK;
}

int lion_set_bodies(lion_sim* s, const int32_t* body_id) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (s->batched) return fail(s, LION_ERR_UNSUPPORTED, "rigid-body exclusion is for single traps");
    const int64_t n = s->n, np = s->d.n_pad;
    bool any = false;
    if (body_id) {
        for (int64_t i = 0; i < n; ++i) {
            if (body_id[i] < -1) return fail(s, LION_ERR_ARG, "body ids must be >= -1");
            any = any || body_id[i] >= 0;
        }
    }
    // pair-once kernels: a tile pair inside one body is skipped whole; tiles of
    // one body only ("aligned" when every tile is such or free) need no per-pair
    // test, other tile pairs whose body-id ranges meet take it
    const int nb = lion::sym_tiles(n);
    std::vector<int32_t> tb(np / 256, -1), tmin(np / 256, INT32_MAX), tmax(np / 256, -1);
    bool aligned = any;
    for (int t = 0; t < nb && any; ++t) {
        const int64_t lo = (int64_t)t * 256, hi = std::min<int64_t>(n, lo + 256);
        bool pure = body_id[lo] >= 0;
        for (int64_t i = lo; i < hi; ++i) {
            pure = pure && body_id[i] == body_id[lo];
            if (body_id[i] >= 0) {
                tmin[t] = std::min(tmin[t], body_id[i]);
                tmax[t] = std::max(tmax[t], body_id[i]);
            }
        }
        tb[t] = pure ? body_id[lo] : -1;
        aligned = aligned && (pure || tmax[t] < 0);
    }
    LION_HIP(s, hipSetDevice(s->device));
    (void)hipStreamSynchronize(s->stream);
    clear_graphs(s);  // captured launches carry the mask pointers
    rigid_off(s);
    if (!any) {
        s->has_bodies = false;
        s->tile_bodies = false;
        s->d.body_code = s->d.body_gmin = s->d.body_gmax = s->d.tile_body = nullptr;
        s->d.tile_bmin = s->d.tile_bmax = nullptr;
        default_shape(s);
        return s->state_set ? refresh_accel(s) : LION_OK;
    }
    std::vector<int32_t> code(np), gmin(np / 16, 0x7fffffff), gmax(np / 16, -1);
    for (int64_t i = 0; i < np; ++i) {
        const int32_t b = i < n ? body_id[i] : -1;
        code[i] = b >= 0 ? b : (int32_t)(-1 - i);
        if (b >= 0) {
            gmin[i / 16] = std::min(gmin[i / 16], b);
            gmax[i / 16] = std::max(gmax[i / 16], b);
        }
    }
    int32_t* dc = (int32_t*)(s->ws + s->body_off[0]);
    int32_t* dmin = (int32_t*)(s->ws + s->body_off[1]);
    int32_t* dmax = (int32_t*)(s->ws + s->body_off[2]);
    hipStream_t st = s->stream;
    LION_HIP(s, hipMemcpyAsync(dc, code.data(), np * 4, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipMemcpyAsync(dmin, gmin.data(), np / 16 * 4, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipMemcpyAsync(dmax, gmax.data(), np / 16 * 4, hipMemcpyHostToDevice, st));
    int32_t* dtb = (int32_t*)(s->ws + s->body_off[3]);
    int32_t* dtr = (int32_t*)(s->ws + s->body_off[4]);
    LION_HIP(s, hipMemcpyAsync(dtb, tb.data(), np / 256 * 4, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipMemcpyAsync(dtr, tmin.data(), np / 256 * 4, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipMemcpyAsync(dtr + np / 256, tmax.data(), np / 256 * 4, hipMemcpyHostToDevice, st));
    LION_HIP(s, hipStreamSynchronize(st));
    s->d.body_code = dc;
    s->d.body_gmin = dmin;
    s->d.body_gmax = dmax;
    s->d.tile_body = dtb;
    s->d.tile_bmin = dtr;
    s->d.tile_bmax = dtr + np / 256;
    s->tile_bodies = aligned;
    s->has_bodies = true;
    default_shape(s);
    return s->state_set ? refresh_accel(s) : LION_OK;
}

int lion_set_rigid_bodies(lion_sim* s, const int32_t* body_id) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (s->batched) return fail(s, LION_ERR_UNSUPPORTED, "rigid bodies are for single traps");
    if (body_id && !s->state_set) return fail(s, LION_ERR_STATE, "set the state before the bodies");
    int rc = lion_set_bodies(s, body_id);  // exclusion mask; turns rigid integration off
    if (rc) return rc;
    if (!s->has_bodies) return LION_OK;
    s->rigid_ids.assign(body_id, body_id + s->n);
    s->rigid_on = true;
    rc = rigid_setup(s);
    if (rc) {
        rigid_off(s);
        return rc;
    }
    return LION_OK;
}

int lion_get_rigid_state(lion_sim* s, int32_t* nbodies, double* com, double* com_velocity,
                         double* angular_momentum, double* quaternion) {
    if (check_handle(s) || !nbodies) return fail(s, LION_ERR_ARG, "null output pointer");
    *nbodies = s->d.nbodies;
    if (s->d.nbodies == 0) return LION_OK;
    std::vector<lion::RigidDev> b(s->d.nbodies);
    LION_HIP(s, hipSetDevice(s->device));
    LION_HIP(s, hipMemcpyAsync(b.data(), s->d.rigid, b.size() * sizeof(lion::RigidDev),
                               hipMemcpyDeviceToHost, s->stream));
    LION_HIP(s, hipStreamSynchronize(s->stream));
    for (size_t k = 0; k < b.size(); ++k)
        for (int c = 0; c < 4; ++c) {
            if (c < 3 && com) com[3 * k + c] = b[k].R[c];
            if (c < 3 && com_velocity) com_velocity[3 * k + c] = b[k].V[c];
            if (c < 3 && angular_momentum) angular_momentum[3 * k + c] = b[k].L[c];
            if (quaternion) quaternion[4 * k + c] = b[k].q[c];
        }
    return LION_OK;
}

int lion_set_species(lion_sim* s, const int32_t* species) {
    if (check_handle(s)) return LION_ERR_ARG;
    const int64_t n = s->n, np = s->d.n_pad;
    std::vector<int32_t> sp(np, 0);
    if (species) {
        for (int64_t i = 0; i < n; ++i) {
            if (species[i] < 0) return fail(s, LION_ERR_ARG, "species labels must be >= 0");
            sp[i] = species[i];
        }
    }
    LION_HIP(s, hipSetDevice(s->device));
    LION_HIP(s, hipMemcpyAsync(s->d.species, sp.data(), np * 4, hipMemcpyHostToDevice, s->stream));
    LION_HIP(s, hipStreamSynchronize(s->stream));
    return LION_OK;
}

int lion_set_beam(lion_sim* s, int32_t beam, int32_t species, double kx, double ky, double kz,
                  double gamma) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (beam < 0 || beam >= lion::kMaxBeams) return fail(s, LION_ERR_ARG, "beam index must be 0..3");
    if (species < -1) return fail(s, LION_ERR_ARG, "species must be >= -1");
    if (!is_fin(kx) || !is_fin(ky) || !is_fin(kz) || !is_fin(gamma) || gamma < 0.0)
        return fail(s, LION_ERR_ARG, "beam direction must be finite and gamma finite and >= 0");
    const double norm = std::sqrt(kx * kx + ky * ky + kz * kz);
    if (gamma > 0.0 && !(norm > 0.0)) return fail(s, LION_ERR_ARG, "beam direction is zero");
    auto& B = s->beams[beam];
    B.gamma = gamma;
    B.species = species;
    B.kx = gamma > 0.0 ? kx / norm : 0.0;
    B.ky = gamma > 0.0 ? ky / norm : 0.0;
    B.kz = gamma > 0.0 ? kz / norm : 0.0;
    return LION_OK;
}

int lion_set_bath(lion_sim* s, int32_t bath, int32_t species, double temperature_K,
                  double damping_time_s, uint64_t seed) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (bath < 0 || bath >= lion::kMaxBaths) return fail(s, LION_ERR_ARG, "bath index must be 0..3");
    if (species < -1) return fail(s, LION_ERR_ARG, "species must be >= -1");
    if (!is_fin(temperature_K) || temperature_K < 0.0 || !is_fin(damping_time_s) ||
        damping_time_s < 0.0)
        return fail(s, LION_ERR_ARG, "temperature and damping time must be finite and >= 0");
    auto& T = s->baths[bath];
    T.temperature = temperature_K;
    T.tau = damping_time_s;
    T.seed = seed;
    T.species = species;
    return LION_OK;
}

int lion_set_step_index(lion_sim* s, int64_t steps_done) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (steps_done < 0) return fail(s, LION_ERR_ARG, "steps_done must be >= 0");
    s->steps_done = steps_done;
    return LION_OK;
}

int64_t lion_get_step_index(const lion_sim* s) { return s ? s->steps_done : -1; }

int lion_set_time_average(lion_sim* s, int32_t window_steps) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (window_steps < 0) return fail(s, LION_ERR_ARG, "window_steps must be >= 0");
    s->avg_window = window_steps;
    s->avg_origin = s->steps_done;
    const int64_t np = s->d.n_pad;
    LION_HIP(s, hipSetDevice(s->device));
    LION_HIP(s, hipMemsetAsync(s->d.vacc, 0, 3 * np * 8, s->stream));
    LION_HIP(s, hipMemsetAsync(s->d.vavg, 0, 3 * np * 8, s->stream));
    LION_HIP(s, hipStreamSynchronize(s->stream));
    return LION_OK;
}

int lion_get_time_average(lion_sim* s, double* vx, double* vy, double* vz,
                          int64_t* window_end_step) {
    if (check_handle(s) || !vx || !vy || !vz || !window_end_step)
        return fail(s, LION_ERR_ARG, "null output pointer");
    if (s->avg_window <= 0) return fail(s, LION_ERR_STATE, "time averaging is off");
    const int64_t done = s->steps_done - s->avg_origin;
    if (done < s->avg_window) return fail(s, LION_ERR_STATE, "no averaging window completed yet");
    const int64_t n = s->n, np = s->d.n_pad;
    LION_HIP(s, hipSetDevice(s->device));
    LION_HIP(s, hipMemcpyAsync(vx, s->d.vavg, n * 8, hipMemcpyDeviceToHost, s->stream));
    LION_HIP(s, hipMemcpyAsync(vy, s->d.vavg + np, n * 8, hipMemcpyDeviceToHost, s->stream));
    LION_HIP(s, hipMemcpyAsync(vz, s->d.vavg + 2 * np, n * 8, hipMemcpyDeviceToHost, s->stream));
    LION_HIP(s, hipStreamSynchronize(s->stream));
    *window_end_step = s->avg_origin + (done / s->avg_window) * s->avg_window;
    return LION_OK;
}

int lion_set_damping(lion_sim* s, int32_t trap, double gamma) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (trap < -1 || trap >= s->n_traps) return fail(s, LION_ERR_ARG, "trap index out of range");
    if (!is_fin(gamma) || gamma < 0.0) return fail(s, LION_ERR_ARG, "gamma must be finite and >= 0");
    const int lo = trap < 0 ? 0 : trap, hi = trap < 0 ? s->n_traps : trap + 1;
    for (int k = lo; k < hi; ++k) s->traps[k].gamma = gamma;
    return LION_OK;
}

static int step_common(lion_sim* s, int64_t nsteps, const double* dts) {
    if (nsteps < 0) return fail(s, LION_ERR_ARG, "nsteps must be >= 0");
    for (int k = 0; k < s->n_traps; ++k)
        if (!is_fin(dts[k]) || dts[k] <= 0.0) return fail(s, LION_ERR_ARG, "dt must be finite and > 0");
    if (!s->state_set) return fail(s, LION_ERR_STATE, "lion_set_state has not been called");
    if (nsteps == 0) return LION_OK;
    LION_HIP(s, hipSetDevice(s->device));
    for (int k = 0; k < s->n_traps; ++k) {
        TrapDev& T = s->traps[k];
        T.dt = dts[k];
        T.h = 0.5 * dts[k];
        T.f = std::exp(-(T.gamma * dts[k]) * 0.5);
        T.t_start = s->t_now[k];
    }
    int rc = upload_traps(s);
    if (rc) return rc;
    bool cooling = false;
    for (const auto& B : s->beams) cooling = cooling || B.gamma > 0.0;
    for (const auto& T : s->baths) cooling = cooling || T.tau > 0.0;
    for (int k = 1; k < s->n_traps && cooling; ++k)
        if (dts[k] != dts[0])
            return fail(s, LION_ERR_UNSUPPORTED, "cooling beams and baths need one dt for all traps");
    rc = upload_cooling(s, dts[0]);
    if (rc) return rc;
    LION_HIP(s, hipMemsetAsync(s->d.counter, 0, sizeof(int64_t), s->stream));
    const int64_t S = chunk_len(s);
    for (int64_t done = 0; done < nsteps;) {
        const int64_t L = std::min(S, nsteps - done);
        rc = run_chunk(s, L);
        if (rc) return rc;
        done += L;
    }
    for (int k = 0; k < s->n_traps; ++k) s->t_now[k] = s->traps[k].t_start + (double)nsteps * dts[k];
    s->steps_done += nsteps;
    return LION_OK;
}

int lion_step(lion_sim* s, int64_t nsteps, double dt) {
    if (check_handle(s)) return LION_ERR_ARG;
    std::vector<double> dts(s->n_traps, dt);
    return step_common(s, nsteps, dts.data());
}

int lion_step_batch(lion_sim* s, int64_t nsteps, const double* dt_per_trap) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (!dt_per_trap) return fail(s, LION_ERR_ARG, "dt_per_trap is NULL");
    return step_common(s, nsteps, dt_per_trap);
}

int lion_prepare_step(lion_sim* s, int64_t nsteps) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (nsteps < 0) return fail(s, LION_ERR_ARG, "nsteps must be >= 0");
    if (nsteps == 0 || s->cfg.use_graph == 2) return LION_OK;
    LION_HIP(s, hipSetDevice(s->device));
    const bool on = cooling_on(s);
    if (on != s->ls.cool_on) {
        LION_HIP(s, hipStreamSynchronize(s->stream));  // no launch of a graph still pending
        clear_graphs(s);
        s->ls.cool_on = on;
    }
    const int64_t S = chunk_len(s);
    hipGraphExec_t ex = nullptr;
    if (nsteps >= S) {
        int rc = chunk_graph(s, S, &ex);
        if (rc) return rc;
    }
    if (nsteps % S) {
        int rc = chunk_graph(s, nsteps % S, &ex);
        if (rc) return rc;
    }
    return LION_OK;
}

int lion_get_state(const lion_sim* cs, double* x, double* y, double* z, double* vx, double* vy,
                   double* vz, double* t) {
    lion_sim* s = const_cast<lion_sim*>(cs);
    if (check_handle(s)) return LION_ERR_ARG;
    const int64_t n = s->n;
    LION_HIP(s, hipSetDevice(s->device));
    std::vector<double4> src(n);
    hipStream_t st = s->stream;
    LION_HIP(s, hipMemcpyAsync(src.data(), s->d.src, n * sizeof(double4), hipMemcpyDeviceToHost, st));
    if (vx) LION_HIP(s, hipMemcpyAsync(vx, s->d.vx, n * 8, hipMemcpyDeviceToHost, st));
    if (vy) LION_HIP(s, hipMemcpyAsync(vy, s->d.vy, n * 8, hipMemcpyDeviceToHost, st));
    if (vz) LION_HIP(s, hipMemcpyAsync(vz, s->d.vz, n * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; ++i) {
        if (x) x[i] = src[i].x;
        if (y) y[i] = src[i].y;
        if (z) z[i] = src[i].z;
    }
    if (t) *t = s->t_now[0];
    return LION_OK;
}

int lion_compute_accel(lion_sim* s, double* ax, double* ay, double* az) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (!ax || !ay || !az) return fail(s, LION_ERR_ARG, "output array is NULL");
    if (!s->state_set) return fail(s, LION_ERR_STATE, "lion_set_state has not been called");
    LION_HIP(s, hipSetDevice(s->device));
    int rc = refresh_accel(s);
    if (rc) return rc;
    const int64_t n = s->n;
    hipStream_t st = s->stream;
    LION_HIP(s, hipMemcpyAsync(ax, s->d.ax, n * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipMemcpyAsync(ay, s->d.ay, n * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipMemcpyAsync(az, s->d.az, n * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipStreamSynchronize(st));
    return LION_OK;
}

size_t lion_normal_modes_workspace_bytes(lion_sim* s) {
    if (check_handle(s) || s->n < 1 || 3 * s->n > 2147483647 / (3 * s->n)) return 0;
    if (hipSetDevice(s->device) != hipSuccess || modes_handle(s) != LION_OK) return 0;
    const int m = (int)(3 * s->n);
    // sizes only: the solver is asked in query mode, with device addresses of
    // the handle's own workspace standing in for the arrays
    double* any = (double*)s->ws;
    size_t scratch = 0;
    std::string err;
    if (lion::eigh_scratch_bytes(s->eigh, m, true, any, any, any, (int*)s->ws, &scratch, err) != 0) {
        s->err = err;
        return 0;
    }
    return modes_fixed_bytes(s->n) + align_up(scratch);
}

int lion_normal_modes(lion_sim* s, void* dev_work, size_t bytes, double* omega2, double* modes) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (!omega2) return fail(s, LION_ERR_ARG, "omega2 output is NULL");
    if (s->batched) return fail(s, LION_ERR_UNSUPPORTED, "normal modes are for single traps");
    if (!s->state_set) return fail(s, LION_ERR_STATE, "lion_set_state has not been called");
    if (s->has_bodies) return fail(s, LION_ERR_UNSUPPORTED, "normal modes with rigid bodies");
    const TrapDev& T = s->traps[0];
    if (T.ps == 0.0 && T.a_rf != 0.0)
        return fail(s, LION_ERR_UNSUPPORTED,
                    "normal modes need a static trap (pseudopotential trap or no rf)");
    if (3 * s->n > 2147483647 / (3 * s->n))
        return fail(s, LION_ERR_UNSUPPORTED, "too many ions for one dense eigen-problem");
    const size_t fixed = modes_fixed_bytes(s->n);
    int rc = check_ws(s, dev_work, bytes, fixed);
    if (rc) return rc;
    LION_HIP(s, hipSetDevice(s->device));
    rc = modes_handle(s);
    if (rc) return rc;
    const int m = (int)(3 * s->n);
    char* base = (char*)dev_work;
    double* A = (double*)base;
    double* W = (double*)(base + align_up((size_t)m * m * 8));
    double* E = (double*)(base + align_up((size_t)m * m * 8) + align_up((size_t)m * 8));
    int* info = (int*)(base + align_up((size_t)m * m * 8) + 2 * align_up((size_t)m * 8));
    std::string err;
    size_t scratch = 0;
    if (lion::eigh_scratch_bytes(s->eigh, m, modes != nullptr, A, W, E, info, &scratch, err) != 0)
        return fail(s, LION_ERR_HIP, err);
    if (bytes < fixed + scratch)
        return fail(s, LION_ERR_WORKSPACE,
                    "normal-mode workspace too small: need " + std::to_string(fixed + scratch) +
                        " bytes (lion_normal_modes_workspace_bytes), got " + std::to_string(bytes));
    hipStream_t st = s->stream;
    LION_HIP(s, lion::launch_hessian(s->d, T, A, st));
    if (lion::eigh_device(s->eigh, A, m, W, E, info, modes != nullptr, base + fixed,
                          bytes - fixed, st, err) != 0)
        return fail(s, LION_ERR_HIP, err);
    int info_h = 0;
    LION_HIP(s, hipMemcpyAsync(omega2, W, (size_t)m * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipMemcpyAsync(&info_h, info, sizeof(int), hipMemcpyDeviceToHost, st));
    if (modes) LION_HIP(s, hipMemcpyAsync(modes, A, (size_t)m * m * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipStreamSynchronize(st));
    if (info_h != 0) return fail(s, LION_ERR_HIP, "eigen-solver did not converge");
    return LION_OK;
}

int lion_minimize(lion_sim* s, double dt, double dmax, double ftol, int64_t max_iter,
                  int64_t* iterations, double* fmax) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (s->batched) return fail(s, LION_ERR_UNSUPPORTED, "minimisation is for single traps");
    if (!s->state_set) return fail(s, LION_ERR_STATE, "lion_set_state has not been called");
    if (s->d.nbodies > 0) return fail(s, LION_ERR_UNSUPPORTED, "minimisation with rigid bodies");
    if (!is_fin(dt) || dt <= 0.0 || !is_fin(dmax) || dmax <= 0.0 || !is_fin(ftol) || ftol < 0.0 ||
        max_iter < 0)
        return fail(s, LION_ERR_ARG, "need dt > 0, dmax > 0, ftol >= 0, max_iter >= 0 (all finite)");
    const TrapDev& T = s->traps[0];
    if (T.ps == 0.0 && T.a_rf != 0.0)
        return fail(s, LION_ERR_UNSUPPORTED,
                    "minimisation needs a time-independent trap (pseudopotential trap or no rf)");
    LION_HIP(s, hipSetDevice(s->device));
    int rc = refresh_accel(s);  // forces at the current positions, trap clock fixed
    if (rc) return rc;
    lion::MinDev m{};
    m.dt = dt;
    m.dmax = dmax;
    m.ftol = ftol;
    m.max_iter = max_iter;
    hipStream_t st = s->stream;
    LION_HIP(s, hipMemcpyAsync(s->d.minst, &m, sizeof(m), hipMemcpyHostToDevice, st));
    const int64_t K = 50;
    for (;;) {
        rc = run_min_chunk(s, K);
        if (rc) return rc;
        LION_HIP(s, hipMemcpyAsync(&m, s->d.minst, sizeof(m), hipMemcpyDeviceToHost, st));
        LION_HIP(s, hipStreamSynchronize(st));
        if (m.done) break;
    }
    if (iterations) *iterations = m.iterations;
    if (fmax) *fmax = m.fmax;
    return LION_OK;
}

int lion_get_energy(lion_sim* s, double* kinetic, double* coulomb, double* dc_trap) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (!s->state_set) return fail(s, LION_ERR_STATE, "lion_set_state has not been called");
    LION_HIP(s, hipSetDevice(s->device));
    const int64_t n = s->n;
    hipStream_t st = s->stream;
    LION_HIP(s, lion::launch_coulomb_potential(s->d, s->n_traps, st));
    std::vector<double> pe(n), vx(n), vy(n), vz(n);
    std::vector<double4> src(n);
    LION_HIP(s, hipMemcpyAsync(pe.data(), s->d.scratch, n * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipMemcpyAsync(src.data(), s->d.src, n * sizeof(double4), hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipMemcpyAsync(vx.data(), s->d.vx, n * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipMemcpyAsync(vy.data(), s->d.vy, n * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipMemcpyAsync(vz.data(), s->d.vz, n * 8, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipStreamSynchronize(st));
    // compensated host sums
    auto add = [](double& sum, double& c, double v) {
        double t = sum + v;
        c += std::fabs(sum) >= std::fabs(v) ? (sum - t) + v : (v - t) + sum;
        sum = t;
    };
    const double ke_e2 = lion::kElementaryCharge * lion::kElementaryCharge / (4.0 * lion::kPi * lion::kEps0);
    double K = 0, Kc = 0, C = 0, Cc = 0, D = 0, Dc = 0;
    for (int k = 0; k < s->n_traps; ++k) {
        const double a_dc = s->traps[k].a_dc, ps = s->traps[k].ps;
        for (int64_t i = s->offsets[k]; i < s->offsets[k + 1]; ++i) {
            const double m = s->mass[i], q = s->charge[i];
            add(K, Kc, 0.5 * m * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]));
            add(C, Cc, 0.5 * ke_e2 * (q / lion::kElementaryCharge) * pe[i]);
            const double4 p = src[i];
            add(D, Dc, q * a_dc * (p.z * p.z - 0.5 * (p.x * p.x + p.y * p.y)));
            if (ps != 0.0) add(D, Dc, 0.5 * q * (q / m) * ps * (p.x * p.x + p.y * p.y));
        }
    }
    if (kinetic) *kinetic = K + Kc;
    if (coulomb) *coulomb = C + Cc;
    if (dc_trap) *dc_trap = D + Dc;
    return LION_OK;
}

int lion_check_finite(lion_sim* s) {
    if (check_handle(s)) return LION_ERR_ARG;
    LION_HIP(s, hipSetDevice(s->device));
    hipStream_t st = s->stream;
    int32_t flags[4] = {0, 0, 0, 0};
    LION_HIP(s, hipMemsetAsync(s->d.flags, 0, 16, st));
    LION_HIP(s, lion::launch_check_finite(s->d, st));
    LION_HIP(s, hipMemcpyAsync(flags, s->d.flags, 16, hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipStreamSynchronize(st));
    if (flags[0] != 0)
        return fail(s, LION_ERR_NONFINITE, std::to_string(flags[0]) + " ions have a non-finite state");
    return LION_OK;
}

int lion_count_lost(lion_sim* s, double r_lost_m, int64_t* count) {
    if (check_handle(s)) return LION_ERR_ARG;
    if (!count) return fail(s, LION_ERR_ARG, "count is NULL");
    if (!(r_lost_m > 0.0) || !std::isfinite(r_lost_m))
        return fail(s, LION_ERR_ARG, "r_lost must be > 0 and finite");
    LION_HIP(s, hipSetDevice(s->device));
    hipStream_t st = s->stream;
    int32_t lost = 0;
    LION_HIP(s, hipMemsetAsync(s->d.flags + 1, 0, sizeof(int32_t), st));
    LION_HIP(s, lion::launch_count_lost(s->d, r_lost_m, st));
    LION_HIP(s, hipMemcpyAsync(&lost, s->d.flags + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LION_HIP(s, hipStreamSynchronize(st));
    *count = lost;
    return LION_OK;
}

const char* lion_last_error(const lion_sim* s) {
    if (!s) return g_create_err.empty() ? "invalid handle" : g_create_err.c_str();
    return s->err.c_str();
}

void lion_destroy(lion_sim* s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    clear_graphs(s);
    lion::eigh_handle_destroy(s->eigh);  // after the synchronisation: no solver work pending
    if (s->capture) (void)hipStreamDestroy(s->capture);
    delete s;
}

int lion_set_kernel_config(lion_sim* s, const lion_kernel_config* c) {
    if (check_handle(s) || !c) return LION_ERR_ARG;
    auto in = [](int v, std::initializer_list<int> set) {
        return v <= 0 || std::find(set.begin(), set.end(), v) != set.end();
    };
    if (!in(c->i_per_lane, {1, 2, 4})) return fail(s, LION_ERR_ARG, "i_per_lane must be 1, 2 or 4");
    if (c->j_split > 64) return fail(s, LION_ERR_ARG, "j_split must be <= 64");
    if (c->chunk_steps > 1000) return fail(s, LION_ERR_ARG, "chunk_steps must be <= 1000");
    if (!in(c->flush_len, {4, 8, 16})) return fail(s, LION_ERR_ARG, "flush_len must be 4, 8 or 16");
    if (!in(c->batch_block, {64, 256, 512, 1024}))
        return fail(s, LION_ERR_ARG, "batch_block must be 64, 256, 512 or 1024");
    if (c->batch_block == 64 && (s->batched ? s->max_trap : s->n) > 64)
        return fail(s, LION_ERR_ARG, "batch_block 64 takes traps of at most 64 ions");
    if (!in(c->use_graph, {1, 2})) return fail(s, LION_ERR_ARG, "use_graph must be 1 or 2");
    if (!in(c->lds_sources, {1, 2})) return fail(s, LION_ERR_ARG, "lds_sources must be 1 or 2");
    if (!in(c->symmetric, {1, 2})) return fail(s, LION_ERR_ARG, "symmetric must be 1 or 2");
    if (!in(c->sym_variant, {1, 2, 3, 4, 5, 6, 7, 8, 9}))
        return fail(s, LION_ERR_ARG, "sym_variant must be 1..9");
    if (!in(c->update_waves, {4, 8, 16})) return fail(s, LION_ERR_ARG, "update_waves must be 4, 8 or 16");
    if (!in(c->small_trap, {1, 2})) return fail(s, LION_ERR_ARG, "small_trap must be 1 or 2");
    if (!in(c->batch_tpt, {1, 2, 4})) return fail(s, LION_ERR_ARG, "batch_tpt must be 1, 2 or 4");
    if (!in(c->step_launches, {1, 2}))
        return fail(s, LION_ERR_ARG, "step_launches must be 1 or 2");
    if (c->symmetric == 2 && (s->batched || lion::sym_tiles(s->n) > lion::kMaxSymTiles))
        return fail(s, LION_ERR_UNSUPPORTED, "pair-once kernels need one trap of N <= 131072");
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    clear_graphs(s);
    s->cfg.i_per_lane = c->i_per_lane;
    s->cfg.j_split = c->j_split;
    s->cfg.flush_len = c->flush_len;
    s->cfg.batch_block = c->batch_block;
    s->cfg.chunk_steps = c->chunk_steps > 0 ? c->chunk_steps : 0;
    s->cfg.use_graph = c->use_graph > 0 ? c->use_graph : 1;
    s->cfg.lds_sources = c->lds_sources;
    s->cfg.symmetric = c->symmetric;
    s->cfg.sym_variant = c->sym_variant;
    s->cfg.update_waves = c->update_waves;
    s->cfg.small_trap = c->small_trap;
    s->cfg.batch_tpt = c->batch_tpt;
    s->cfg.step_launches = c->step_launches;
    default_shape(s);
    return LION_OK;
}

int lion_get_kernel_config(const lion_sim* s, lion_kernel_config* c) {
    if (check_handle(s) || !c) return LION_ERR_ARG;
    c->i_per_lane = s->ls.i_per_lane;
    c->j_split = s->ls.j_split;
    c->chunk_steps = (int32_t)chunk_len(s);
    c->flush_len = s->ls.flush_len;
    c->batch_block = s->ls.batch_block;
    c->use_graph = s->cfg.use_graph;
    c->lds_sources = s->ls.lds_sources ? 2 : 1;
    c->symmetric = s->ls.symmetric ? 2 : 1;
    c->sym_variant = s->ls.sym_variant + 1;
    c->update_waves = s->ls.update_waves;
    c->small_trap = s->ls.small_path ? 2 : 1;
    c->batch_tpt = s->ls.batch_tpt;
    c->step_launches = rows_active(s) ? 1 : 2;
    return LION_OK;
}

int lion_time_pair_kernel(lion_sim* s, int32_t reps, double* ms_avg) {
    if (check_handle(s) || !ms_avg) return LION_ERR_ARG;
    if (s->batched) return fail(s, LION_ERR_UNSUPPORTED, "single-trap handles only");
    if (reps < 1 || reps > 10000) return fail(s, LION_ERR_ARG, "reps must be 1..10000");
    if (!s->state_set) return fail(s, LION_ERR_STATE, "lion_set_state has not been called");
    LION_HIP(s, hipSetDevice(s->device));
    hipStream_t st = s->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LION_HIP(s, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(s, LION_ERR_HIP, "hipEventCreate failed");
    }
    // one warm launch, then reps back-to-back launches between two events
    int rc = lion::launch_pair(s->d, s->precision, s->ls, false, st) == hipSuccess ? LION_OK
             : fail(s, LION_ERR_HIP, "pair kernel launch failed");
    if (rc == LION_OK && hipEventRecord(e0, st) != hipSuccess) rc = fail(s, LION_ERR_HIP, "hipEventRecord failed");
    for (int r = 0; r < reps && rc == LION_OK; ++r)
        if (lion::launch_pair(s->d, s->precision, s->ls, false, st) != hipSuccess)
            rc = fail(s, LION_ERR_HIP, "pair kernel launch failed");
    if (rc == LION_OK && hipEventRecord(e1, st) != hipSuccess) rc = fail(s, LION_ERR_HIP, "hipEventRecord failed");
    float ms = 0.0f;
    if (rc == LION_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(s, LION_ERR_HIP, "hipEventSynchronize failed");
    if (rc == LION_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        rc = fail(s, LION_ERR_HIP, "hipEventElapsedTime failed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == LION_OK) *ms_avg = (double)ms / reps;
    return rc;
}

int lion_time_batch_kernel(lion_sim* s, int32_t reps, int32_t nsteps, double dt, double* ms_avg) {
    if (check_handle(s) || !ms_avg) return LION_ERR_ARG;
    if (!s->batched) return fail(s, LION_ERR_UNSUPPORTED, "batched handles only");
    if (reps < 1 || reps > 10000 || nsteps < 1 || nsteps > 100000)
        return fail(s, LION_ERR_ARG, "reps must be 1..10000 and nsteps 1..100000");
    std::vector<double> dts(s->n_traps, dt);
    // set up clocks, step sizes and damping factors exactly as lion_step does
    int rc = step_common(s, 0, dts.data());
    if (rc) return rc;
    if (!is_fin(dt) || dt <= 0.0) return fail(s, LION_ERR_ARG, "dt must be finite and > 0");
    for (int k = 0; k < s->n_traps; ++k) {
        TrapDev& T = s->traps[k];
        T.dt = dt;
        T.h = 0.5 * dt;
        T.f = std::exp(-(T.gamma * dt) * 0.5);
        T.t_start = s->t_now[k];
    }
    rc = upload_traps(s);
    if (rc) return rc;
    rc = upload_cooling(s, dt);
    if (rc) return rc;
    hipStream_t st = s->stream;
    LION_HIP(s, hipMemsetAsync(s->d.counter, 0, sizeof(int64_t), st));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LION_HIP(s, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(s, LION_ERR_HIP, "hipEventCreate failed");
    }
    if (hipEventRecord(e0, st) != hipSuccess) rc = fail(s, LION_ERR_HIP, "hipEventRecord failed");
    for (int r = 0; r < reps && rc == LION_OK; ++r) {
        if (lion::launch_batch(s->d, s->precision, s->n_traps, s->max_trap, s->ls, nsteps, 0, st) != hipSuccess ||
            lion::launch_counter_add(s->d, nsteps, st) != hipSuccess)
            rc = fail(s, LION_ERR_HIP, "batch kernel timing launch failed");
    }
    if (rc == LION_OK && hipEventRecord(e1, st) != hipSuccess) rc = fail(s, LION_ERR_HIP, "hipEventRecord failed");
    float ms = 0.0f;
    if (rc == LION_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(s, LION_ERR_HIP, "hipEventSynchronize failed");
    if (rc == LION_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        rc = fail(s, LION_ERR_HIP, "hipEventElapsedTime failed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LION_OK) return rc;
    const double total = ms;
    for (int k = 0; k < s->n_traps; ++k)
        s->t_now[k] = s->traps[k].t_start + (double)((int64_t)reps * nsteps) * dt;
    s->steps_done += (int64_t)reps * nsteps;
    *ms_avg = total / reps;
    return LION_OK;
}

int lion_mathieu_to_voltages(double q_x, double a_x, double M, double Q, double Omega, double r0,
                             double z0, double kappa, double* V0, double* U0) {
    if (!V0 || !U0) return LION_ERR_ARG;
    if (!is_fin(q_x) || !is_fin(a_x) || !is_fin(M) || !is_fin(Q) || !is_fin(Omega) ||
        !is_fin(r0) || !is_fin(z0) || !is_fin(kappa))
        return LION_ERR_ARG;
    if (M <= 0 || Q == 0 || Omega <= 0 || r0 <= 0 || z0 <= 0) return LION_ERR_ARG;
    if (a_x != 0.0 && kappa == 0.0) return LION_ERR_ARG;
    // eq. (Mathieuaq): q_x = 2 Q V0 / (M r0^2 Omega^2), a_x = -4 Q kappa U0 / (M z0^2 Omega^2)
    *V0 = q_x * M * r0 * r0 * Omega * Omega / (2.0 * Q);
    *U0 = a_x == 0.0 ? 0.0 : -a_x * M * z0 * z0 * Omega * Omega / (4.0 * Q * kappa);
    return LION_OK;
}

void lion_constants(double* e_charge, double* eps0, double* amu) {
    if (e_charge) *e_charge = lion::kElementaryCharge;
    if (eps0) *eps0 = lion::kEps0;
    if (amu) *amu = lion::kAmu;
}

}  // extern "C"
