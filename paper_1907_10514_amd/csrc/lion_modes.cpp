// Symmetric eigen-decomposition of the mass-weighted Hessian on the GPU with
// rocSOLVER (divide and conquer, dsyevd).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <string>

#include "lion_internal.h"

namespace lion {

int eigh_device(double* A, int m, double* W, double* E, int* info, bool vectors, hipStream_t st,
                std::string& err) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) {
        err = "rocblas_create_handle failed";
        return -1;
    }
    int rc = 0;
    if (rocblas_set_stream(h, st) != rocblas_status_success) {
        err = "rocblas_set_stream failed";
        rc = -1;
    }
    if (rc == 0) {
        const rocblas_status s =
            rocsolver_dsyevd(h, vectors ? rocblas_evect_original : rocblas_evect_none,
                             rocblas_fill_upper, m, A, m, W, E, info);
        if (s != rocblas_status_success) {
            err = std::string("rocsolver_dsyevd: ") + rocblas_status_to_string(s);
            rc = -1;
        }
    }
    (void)rocblas_destroy_handle(h);
    return rc;
}

}  // namespace lion
