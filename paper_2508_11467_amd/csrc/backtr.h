// Back-transformation of singular vectors by blocks of Householder
// reflectors in the modified compact WY form (k_backtr.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bdc {

constexpr int kBtMaxBlock = 64;  // reflectors per block, at most
constexpr int kBtSlices = 8;     // depth slices of the Y^T products, at most

// scratch bytes of launch_backtr for an m x p matrix and block b
size_t backtr_bytes(int m, int p, int block);

// C (m x p, ldc) <- Q C (trans 0) or Q^T C (trans 1), Q = H_0 ... H_{k-1};
// reflector i has its unit pivot at row i + offset, zeros above, and entry r
// below at Y[r * rs + i * cs]; tau[i] = 0 makes H_i the identity
void launch_backtr(int trans, int m, int p, int k, int offset, const double* Y, int64_t rs, int64_t cs,
                   const double* tau, double* C, int ldc, int block, void* scratch, hipStream_t st);

}  // namespace bdc
