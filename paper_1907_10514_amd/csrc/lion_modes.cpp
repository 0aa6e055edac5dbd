// Symmetric eigen-decomposition of the mass-weighted Hessian on the GPU with
// rocSOLVER (divide and conquer, dsyevd).  The solver's scratch memory is
// handed to rocBLAS from the caller's workspace (rocblas_set_workspace), so
// rocBLAS allocates no device memory of its own for it.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <string>

#include "lion_internal.h"

namespace lion {

namespace {

rocblas_evect evect_of(bool vectors) {
    return vectors ? rocblas_evect_original : rocblas_evect_none;
}

}  // namespace

int eigh_handle_create(void** out, std::string& err) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) {
        err = "rocblas_create_handle failed";
        return -1;
    }
    *out = h;
    return 0;
}

void eigh_handle_destroy(void* h) {
    if (h) (void)rocblas_destroy_handle((rocblas_handle)h);
}

int eigh_scratch_bytes(void* hv, int m, bool vectors, double* A, double* W, double* E,
                       int* info, size_t* bytes, std::string& err) {
    rocblas_handle h = (rocblas_handle)hv;
    if (rocblas_start_device_memory_size_query(h) != rocblas_status_success) {
        err = "rocblas_start_device_memory_size_query failed";
        return -1;
    }
    const rocblas_status s =
        rocsolver_dsyevd(h, evect_of(vectors), rocblas_fill_upper, m, A, m, W, E, info);
    size_t size = 0;
    const rocblas_status s2 = rocblas_stop_device_memory_size_query(h, &size);
    if ((s != rocblas_status_success && s != rocblas_status_size_increased &&
         s != rocblas_status_size_unchanged) ||
        s2 != rocblas_status_success) {
        err = std::string("rocsolver_dsyevd size query: ") + rocblas_status_to_string(s);
        return -1;
    }
    *bytes = size;
    return 0;
}

int eigh_device(void* hv, double* A, int m, double* W, double* E, int* info, bool vectors,
                void* scratch, size_t scratch_bytes, hipStream_t st, std::string& err) {
    rocblas_handle h = (rocblas_handle)hv;
    if (rocblas_set_stream(h, st) != rocblas_status_success) {
        err = "rocblas_set_stream failed";
        return -1;
    }
    if (rocblas_set_workspace(h, scratch, scratch_bytes) != rocblas_status_success) {
        err = "rocblas_set_workspace failed";
        return -1;
    }
    const rocblas_status s =
        rocsolver_dsyevd(h, evect_of(vectors), rocblas_fill_upper, m, A, m, W, E, info);
    if (s != rocblas_status_success) {
        err = std::string("rocsolver_dsyevd: ") + rocblas_status_to_string(s);
        return -1;
    }
    return 0;
}

}  // namespace lion
