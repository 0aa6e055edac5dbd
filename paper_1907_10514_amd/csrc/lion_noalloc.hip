// Allocation-free force evaluation: lion_accel_noalloc.
//
// The same accelerations as lion_compute_accel on a single-trap handle, for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid it).  The caller passes device
// inputs and outputs; everything else the kernels need (the packed source
// streams, Q/M per ion, the trap parameters and the per-slice partial sums)
// lives in one file-scope device array of kScratchBytes, which each GPU the
// library runs on holds until the process ends.  Host code addresses that
// array only through the pointer hipGetSymbolAddress returns for the current
// device (taken once per device, on the first call there).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "lion.h"
#include "lion_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(8) << 20;  // 8 MiB per device
constexpr int64_t kMaxIons = 65536;
constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int fail(int code, const std::string& msg) {
    lion::set_handle_free_error("lion_accel_noalloc: " + msg);
    return code;
}

// The device address of `scratch` on the current device.
int scratch_of_current_device(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(LION_ERR_HIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return fail(LION_ERR_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LION_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return LION_OK;
}

bool is_fin(double v) { return std::isfinite(v); }

}  // namespace

extern "C" int lion_accel_noalloc(int64_t n, const double* x, const double* y, const double* z,
                                  const double* charges_C, const double* masses_kg, double V_rf,
                                  double Omega, double U_dc, double r0, double z0, double kappa,
                                  double t, int precision, double* ax, double* ay, double* az,
                                  void* hip_stream) {
    if (n < 1 || n > kMaxIons)
        return fail(LION_ERR_ARG, "n must be 1.." + std::to_string(kMaxIons) +
                                      " (the scratch array holds " +
                                      std::to_string(kScratchBytes) + " bytes)");
    if (precision < LION_FP64 || precision > LION_MIXED_KAHAN)
        return fail(LION_ERR_ARG, "unknown precision");
    if (!x || !y || !z || !charges_C || !masses_kg || !ax || !ay || !az)
        return fail(LION_ERR_ARG, "an input or output pointer is NULL");
    if (!is_fin(V_rf) || !is_fin(Omega) || !is_fin(U_dc) || !is_fin(r0) || !is_fin(z0) ||
        !is_fin(kappa) || !is_fin(t))
        return fail(LION_ERR_ARG, "trap parameter or time not finite");
    if (r0 <= 0 || z0 <= 0) return fail(LION_ERR_ARG, "r0 and z0 must be > 0");
    if (V_rf != 0.0 && Omega <= 0.0) return fail(LION_ERR_ARG, "Omega must be > 0 when V_rf != 0");
    void* base = nullptr;
    int rc = scratch_of_current_device(&base);
    if (rc) return rc;

    // launch shape of the all-pairs kernels, as a single-trap handle picks it,
    // with the source slices limited to what the scratch array holds
    const bool mixed = precision != LION_FP64;
    const int64_t n_pad = round_up(n, 1024);
    const int64_t n64 = round_up(n, 64);
    lion::LaunchShape ls{};
    ls.i_per_lane = n >= 16384 ? (mixed ? 4 : 2) : 1;
    ls.flush_len = 8;
    ls.batch_block = 256;
    ls.lds_sources = 1;
    ls.symmetric = 0;
    ls.update_waves = 4;
    const size_t fixed = align_up(sizeof(lion::TrapDev)) + 2 * align_up(n_pad * 32) +
                         2 * align_up(n_pad * 8);
    const int64_t j_fit = (int64_t)((kScratchBytes - fixed) / align_up(3 * n_pad * 8));
    const int64_t blocks_x = (n + 64 * ls.i_per_lane - 1) / (64 * ls.i_per_lane);
    const int64_t target = n >= 16384 ? 1024 : 4096;
    int64_t j = (target + blocks_x - 1) / blocks_x;
    j = std::max<int64_t>(1, std::min<int64_t>({j, 64, n64 / 64, j_fit}));
    ls.jps = (int)round_up((n64 + j - 1) / j, 64);
    ls.j_split = (int)((n64 + ls.jps - 1) / ls.jps);

    // the arrays of the kernels, carved from the scratch array
    char* p = (char*)base;
    lion::DevState d{};
    d.n = n;
    d.n_pad = n_pad;
    d.traps = (lion::TrapDev*)p;
    p += align_up(sizeof(lion::TrapDev));
    d.src = (double4*)p;
    p += align_up(n_pad * 32);
    d.srcm = mixed ? (lion::MixedSrc*)p : nullptr;
    p += align_up(n_pad * 32);
    d.qm = (double*)p;
    p += align_up(n_pad * 8);
    d.qe = (double*)p;
    p += align_up(n_pad * 8);
    d.part = (double*)p;
    d.ax = ax;
    d.ay = ay;
    d.az = az;

    lion::TrapDev T{};
    T.a_rf = V_rf / (r0 * r0);
    T.omega = Omega;
    T.a_dc = kappa * U_dc / (z0 * z0);
    T.f = 1.0;
    T.t_start = t;
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = lion::launch_pack_inputs(x, y, z, charges_C, masses_kg, d, T, st);
    if (e == hipSuccess) e = lion::launch_pair(d, precision, ls, false, st);
    if (e == hipSuccess) e = lion::launch_update(d, precision, ls, lion::kModeAccel, false, st);
    if (e != hipSuccess) return fail(LION_ERR_HIP, hipGetErrorString(e));
    return LION_OK;
}
