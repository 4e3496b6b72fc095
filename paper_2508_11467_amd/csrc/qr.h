// Householder QR of a tall matrix and its explicit Q (k_qr.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace bdc {

// bytes of the grid-barrier state and the panel's partial sums for up to
// max_wg workgroups
size_t qr_sync_bytes(int max_wg);
// largest panel width
int qr_max_block();
// workgroups and rows per workgroup of the panel kernel for `rows_below`
// rows under a top block of b columns (at most 10240 / b rows per
// workgroup): 0, or 1 when the rows do not fit the resident grid, -1 on a
// runtime error
int qr_panel_grid(int device, int rows_below, int b, int* grid, int* rows_per_wg);

// A (m x n, lda, m >= n) <- R above the diagonal and the reflectors below it,
// tau (n): LAPACK's geqrf storage, panels of b columns.  sync_buf: zeroed
// state of qr_sync_bytes; bt_scratch: backtr_bytes(m, n, b).  Returns BDC_OK,
// BDC_ERR_TOO_LARGE or BDC_ERR_HIP (launches enqueued on st).
int launch_geqrf(int device, int m, int n, double* A, int lda, double* tau, int b, void* sync_buf, size_t sync_bytes,
                 void* bt_scratch, hipStream_t st);

// Q (m x ncols, ldq) <- the first ncols columns of H_0 ... H_{k-1} (geqrf
// storage in A), blocks of b reflectors; bt_scratch: backtr_bytes(m, ncols, b)
void launch_orgqr(int m, int ncols, int k, const double* A, int lda, const double* tau, double* Q, int ldq, int b,
                  void* bt_scratch, hipStream_t st);

}  // namespace bdc
