// Back-transformation of singular vectors by blocks of Householder
// reflectors in the modified compact WY form (k_backtr.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bdc {

constexpr int kBtMaxBlock = 64;  // reflectors per block, at most
constexpr int kBtSlices = 32;    // depth slices of the Y^T products, at most

// the allocation-free entry point: a fixed 32 MiB of device memory per GPU,
// C taken in panels of at most 512 columns
constexpr size_t kBtFixedScratchBytes = size_t(32) << 20;
constexpr int kBtFixedPanel = 512;
constexpr int kBtMaxDevices = 64;

// scratch bytes of launch_backtr for m rows, column panels of `panel`
// columns and blocks of `block` reflectors
size_t backtr_bytes(int m, int panel, int block);

// C (m x p, ldc) <- Q C (trans 0) or Q^T C (trans 1), Q = H_0 ... H_{k-1};
// reflector i has its unit pivot at row i + offset, zeros above, and entry r
// below at Y[r * rs + i * cs]; tau[i] = 0 makes H_i the identity.  The
// columns of C are taken `panel` at a time (every column is transformed on
// its own, so any panel width gives the same results).  The Y^T products
// split their depth into at most kBtSlices slices (enough for about a
// thousand workgroups over p columns), added in a fixed order.
void launch_backtr(int trans, int m, int p, int k, int offset, const double* Y, int64_t rs, int64_t cs,
                   const double* tau, double* C, int ldc, int block, void* scratch, int panel, hipStream_t st);

// C (rows x N, ldc) -= Y (rows x K, ldy) Z (K x N, ldz), column-major, on the
// FP64 matrix cores
void launch_sub_product(int rows, int N, int K, const double* Y, int ldy, const double* Z, int ldz, double* C,
                        int ldc, hipStream_t st);

// device address of the fixed scratch on `device` (which must be current),
// looked up once per device; nullptr if the lookup failed
void* backtr_fixed_scratch(int device);

}  // namespace bdc
