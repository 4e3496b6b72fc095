// Split-precision products on the int8 matrix cores by the Chinese remainder
// theorem (k_crt.hip): buffer layout and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bdc {

constexpr int kCrtMinMod = 13, kCrtMaxMod = 16;  // supported numbers of moduli
constexpr int kCrtMaxBeta = 55;                   // scaled operands are integers of at most 56 bits

// residue planes: k padded to a multiple of 64 (one k stage of the products),
// rows and columns to a multiple of 256 (one output tile)
__host__ __device__ inline int crt_kpad(int K) { return ((K > 0 ? K : 1) + 63) / 64 * 64; }
__host__ __device__ inline int crt_rowpad(int R) { return ((R > 0 ? R : 1) + 255) / 256 * 256; }

// largest beta <= kCrtMaxBeta with P 2^(2 beta) <= (M - 1) / 2 for the first L moduli
int crt_beta(int L, int P);
bool crt_supported(int L);

struct CrtBuffers {
  void* base;
  int8_t* ra;                // L planes of Mp x P residues of A (rows, k contiguous)
  int8_t* rb;                // L planes of Np x P residues of B^T
  int8_t* rc;                // L planes of Mp x N residues of C (column-major, ld Mp)
  unsigned long long* amax;  // per row of A / column of B: bits of the largest |entry|
  unsigned long long* bmax;
  int* ea;                   // scale exponents
  int* eb;
};

// bytes of the buffers of a plain M x N x K product; with b != NULL (b->base
// set) the pointers are laid out from b->base
size_t crt_plain_bytes(int L, int M, int N, int K, CrtBuffers* b);

// C (M x N, ldc) = A (M x K, lda) B (K x N, ldb), column-major FP64
void launch_gemm_crt_plain(int L, int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C,
                           int ldc, const CrtBuffers& b, hipStream_t st);

}  // namespace bdc
