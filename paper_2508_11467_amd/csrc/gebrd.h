// Householder bidiagonal reduction, merged-rank-(2b) form (k_gebrd.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace bdc {

// panel width, at most
int gebrd_max_block();
// bytes of the panel buffers (P: m x 2b, Q^T: 2b x n), the grid-barrier
// state and the partial sums of up to max_wg workgroups
size_t gebrd_work_bytes(int m, int n, int b, int max_wg);
// A (m x n, lda, m >= n) <- d, e, the column reflectors below the diagonal
// and the row reflectors right of the superdiagonal (LAPACK's gebrd
// storage); tauq, taup (n; taup[n-1] = 0), d (n), e (n-1).  Returns BDC_OK,
// BDC_ERR_TOO_LARGE (work too small) or BDC_ERR_HIP.
int launch_gebrd(int device, int m, int n, double* A, int lda, double* tauq, double* taup, double* d, double* e,
                 int b, void* work, size_t work_bytes, int max_wg, hipStream_t st);

}  // namespace bdc
