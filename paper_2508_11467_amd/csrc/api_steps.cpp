// Single-step entry points: each runs one stage of a merge through the same
// kernels as bdc_svd, on a one-node plan built around caller-provided inputs,
// in a temporary workspace.  They synchronise the stream and are meant for
// checking each stage against an independent implementation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "bdc.h"
#include "bdc_internal.h"
#include "crt.h"

using namespace bdc;

namespace {

struct Tmp {
  std::vector<void*> bufs;
  bool ok = true;
  template <class T>
  T* alloc(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
      ok = false;
      return nullptr;
    }
    (void)hipMemset(p, 0, std::max<size_t>(n, 1) * sizeof(T));
    bufs.push_back(p);
    return (T*)p;
  }
  ~Tmp() {
    for (void* p : bufs) (void)hipFree(p);
  }
};

// A workspace for one problem of size n (all per-position arrays length n).
Work make_work(Tmp& t, int64_t n) {
  Work w{};
  const size_t N1 = (size_t)n, N2 = (size_t)(n * n);
  w.Uw = t.alloc<double>(N2);
  w.Vw = t.alloc<double>(N2);
  w.GU = t.alloc<double>(N2);
  w.GV = t.alloc<double>(N2);
  w.UM = t.alloc<double>(N2);
  w.VM = t.alloc<double>(N2);
  w.sig = t.alloc<double>(N1);
  w.ps_d = t.alloc<double>(N1);
  w.ps_z = t.alloc<double>(N1);
  w.sd = t.alloc<double>(N1);
  w.sz = t.alloc<double>(N1);
  w.dval = t.alloc<double>(N1);
  w.tau = t.alloc<double>(N1);
  w.zt = t.alloc<double>(N1);
  w.rot_cs = t.alloc<double>(2 * N1);
  w.col = t.alloc<int32_t>(N1);
  w.ulo = t.alloc<int32_t>(N1);
  w.uhi = t.alloc<int32_t>(N1);
  w.vlo = t.alloc<int32_t>(N1);
  w.vhi = t.alloc<int32_t>(N1);
  w.ps_c = t.alloc<int32_t>(N1);
  w.ps_col = t.alloc<int32_t>(N1);
  w.ps_sup = t.alloc<int32_t>(N1);
  w.status = t.alloc<int32_t>(N1);
  w.ps_rot = t.alloc<int32_t>(N1);
  w.cand = t.alloc<int32_t>(N1);
  w.scol = t.alloc<int32_t>(N1);
  w.srot = t.alloc<int32_t>(N1);
  w.sgrp = t.alloc<int32_t>(N1);
  w.gsurv = t.alloc<int32_t>(N1);
  w.dcol = t.alloc<int32_t>(N1);
  w.drot = t.alloc<int32_t>(N1);
  w.o = t.alloc<int32_t>(N1);
  w.iters = t.alloc<int32_t>(N1);
  w.rot_pos = t.alloc<int32_t>(2 * N1);
  w.rot_col = t.alloc<int32_t>(2 * N1);
  w.st = t.alloc<NodeState>(1);
  w.ctl = t.alloc<Ctl>(1);
  w.leaf_fl = t.alloc<unsigned long long>(1);
  w.sec = t.alloc<SecCount>(1);
  w.oz.min_n = INT32_MAX;
  w.small_n = 96;
  w.sec_small_n = 0;
  w.max_secular_iters = 64;
  w.max_leaf_sweeps = 40;
  return w;
}

struct Guard {
  int old = -1;
  explicit Guard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) old = -1;
    (void)hipSetDevice(dev);
  }
  ~Guard() {
    if (old >= 0) (void)hipSetDevice(old);
  }
};

int finish(hipStream_t st) {
  if (hipGetLastError() != hipSuccess) return BDC_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return BDC_ERR_HIP;
  return BDC_OK;
}

}  // namespace

extern "C" {

int bdc_step_leaf(bdc_handle_t h, int m, int s, const double* d, const double* e, double* sigma,
                  double* W, double* Q, bdc_stream_t stream) {
  int dev, msi, mls;
  if (bdc::handle_info(h, &dev, &msi, &mls) != BDC_OK) return BDC_ERR_INVALID_HANDLE;
  if (m < 1 || m > kMaxLeaf) return -2;
  if (s != 0 && s != 1) return -3;
  if (!d) return -4;
  if (m - 1 + s > 0 && !e) return -5;
  if (!sigma) return -6;
  if (!W) return -7;
  if (!Q) return -8;
  Guard g(dev);
  hipStream_t st = (hipStream_t)stream;
  const int ld = m + s;
  Tmp t;
  Work w = make_work(t, ld);
  LeafDesc* ld_dev = t.alloc<LeafDesc>(1);
  if (!t.ok) return BDC_ERR_NOMEM;
  w.d = d;
  w.e = e;
  w.max_leaf_sweeps = mls;
  LeafDesc L{0, 0, ld, 0, m, s};
  if (hipMemcpy(ld_dev, &L, sizeof(L), hipMemcpyHostToDevice) != hipSuccess) return BDC_ERR_HIP;
  launch_reset(w.ctl, w.st, w.sec, 1, st);
  launch_leaf(ld_dev, 1, m, w, st);
  if (hipMemcpy2DAsync(W, sizeof(double) * m, w.Uw, sizeof(double) * ld, sizeof(double) * m, m,
                       hipMemcpyDeviceToDevice, st) != hipSuccess)
    return BDC_ERR_HIP;
  if (hipMemcpyAsync(Q, w.Vw, sizeof(double) * ld * ld, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return BDC_ERR_HIP;
  if (hipMemcpyAsync(sigma, w.sig, sizeof(double) * m, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return BDC_ERR_HIP;
  return finish(st);
}

int bdc_step_deflate(bdc_handle_t h, int m, int s, const double* sig, const double* qrow1,
                     const double* qrow2, double alpha, double beta, int32_t* perm, double* dz,
                     int32_t* status, int32_t* rot_pos, double* rot_cs, double* misc, int32_t* nrot,
                     bdc_stream_t stream) {
  int dev, msi, mls;
  if (bdc::handle_info(h, &dev, &msi, &mls) != BDC_OK) return BDC_ERR_INVALID_HANDLE;
  if (m < 3) return -2;
  if (s != 0 && s != 1) return -3;
  if (!sig) return -4;
  if (!qrow1) return -5;
  if (!qrow2) return -6;
  if (!std::isfinite(alpha)) return -7;
  if (!std::isfinite(beta)) return -8;
  if (!perm) return -9;
  if (!dz) return -10;
  if (!status) return -11;
  if (!rot_pos) return -12;
  if (!rot_cs) return -13;
  if (!misc) return -14;
  if (!nrot) return -15;
  Guard g(dev);
  hipStream_t st = (hipStream_t)stream;
  const int k = m / 2, ld = m + s;
  Tmp t;
  Work w = make_work(t, ld);
  double* dd = t.alloc<double>(ld);
  double* ee = t.alloc<double>(ld);
  NodeDesc* nd_dev = t.alloc<NodeDesc>(1);
  if (!t.ok) return BDC_ERR_NOMEM;
  w.d = dd;
  w.e = ee;
  // the two rows of the children's right bases the merge reads
  if (hipMemcpy2D(w.Vw + (k - 1), sizeof(double) * ld, qrow1, sizeof(double), sizeof(double), k,
                  hipMemcpyDeviceToDevice) != hipSuccess)
    return BDC_ERR_HIP;
  if (hipMemcpy2D(w.Vw + k + (int64_t)k * ld, sizeof(double) * ld, qrow2, sizeof(double), sizeof(double),
                  m - k + s, hipMemcpyDeviceToDevice) != hipSuccess)
    return BDC_ERR_HIP;
  if (hipMemcpy(w.sig, sig, sizeof(double) * m, hipMemcpyDeviceToDevice) != hipSuccess) return BDC_ERR_HIP;
  std::vector<int32_t> ident(ld), lo(ld, 0), hi(ld, ld);
  for (int i = 0; i < ld; ++i) ident[i] = i;
  std::vector<double> dh(ld, 0.0), eh(ld, 0.0);
  dh[k - 1] = alpha;
  eh[k - 1] = beta;
  NodeDesc nd{0, 0, ld, 0, m, s, k, 0};
  if (hipMemcpy(w.col, ident.data(), sizeof(int32_t) * ld, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(w.vlo, lo.data(), sizeof(int32_t) * ld, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(w.vhi, hi.data(), sizeof(int32_t) * ld, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(w.ulo, lo.data(), sizeof(int32_t) * ld, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(w.uhi, hi.data(), sizeof(int32_t) * ld, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dd, dh.data(), sizeof(double) * ld, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(ee, eh.data(), sizeof(double) * ld, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(nd_dev, &nd, sizeof(nd), hipMemcpyHostToDevice) != hipSuccess)
    return BDC_ERR_HIP;
  launch_reset(w.ctl, w.st, w.sec, 1, st);
  launch_prep(nd_dev, 1, m, w, st);
  int rc = finish(st);
  if (rc != BDC_OK) return rc;
  NodeState ns;
  if (hipMemcpy(&ns, w.st, sizeof(ns), hipMemcpyDeviceToHost) != hipSuccess) return BDC_ERR_HIP;
  const double mh[8] = {ns.scale, ns.tol, ns.c0, ns.s0, (double)ns.N, (double)ns.n1, (double)ns.n2, (double)ns.n3};
  if (hipMemcpy(misc, mh, sizeof(mh), hipMemcpyHostToDevice) != hipSuccess) return BDC_ERR_HIP;
  if (hipMemcpy(nrot, &ns.nrot, sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) return BDC_ERR_HIP;
  if (hipMemcpy(perm, w.ps_c, sizeof(int32_t) * m, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(dz, w.ps_d, sizeof(double) * m, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(dz + m, w.ps_z, sizeof(double) * m, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(status, w.status, sizeof(int32_t) * m, hipMemcpyDeviceToDevice) != hipSuccess)
    return BDC_ERR_HIP;
  if (ns.nrot > 0 &&
      (hipMemcpy(rot_pos, w.rot_pos, sizeof(int32_t) * 2 * ns.nrot, hipMemcpyDeviceToDevice) != hipSuccess ||
       hipMemcpy(rot_cs, w.rot_cs, sizeof(double) * 2 * ns.nrot, hipMemcpyDeviceToDevice) != hipSuccess))
    return BDC_ERR_HIP;
  return BDC_OK;
}

int bdc_step_secular_start(bdc_handle_t h, int N, const double* d, const double* z, const float* xstart,
                           int32_t* o, double* tau, int32_t* iters, bdc_stream_t stream) {
  int dev, msi, mls;
  if (bdc::handle_info(h, &dev, &msi, &mls) != BDC_OK) return BDC_ERR_INVALID_HANDLE;
  if (N < 1) return -2;
  if (!d) return -3;
  if (!z) return -4;
  if (!o) return -6;
  if (!tau) return -7;
  if (!iters) return -8;
  Guard g(dev);
  hipStream_t st = (hipStream_t)stream;
  Tmp t;
  Work w = make_work(t, 1);
  double* sd = t.alloc<double>(N);
  double* sz = t.alloc<double>(N);
  NodeDesc* nd_dev = t.alloc<NodeDesc>(1);
  if (!t.ok) return BDC_ERR_NOMEM;
  w.sd = sd;
  w.sz = sz;
  w.o = o;
  w.tau = tau;
  w.iters = iters;
  w.xs = const_cast<float*>(xstart);  // read only by the secular kernel
  w.max_secular_iters = msi;
  w.sec_small_n = bdc::handle_sec_small(h);
  std::vector<double> zh(N);
  if (hipMemcpy(zh.data(), z, sizeof(double) * N, hipMemcpyDeviceToHost) != hipSuccess) return BDC_ERR_HIP;
  double rho = 0.0;
  for (double v : zh) rho += v * v;
  NodeState ns{};
  ns.N = N;
  ns.rho = rho;
  NodeDesc nd{0, 0, N, 0, N, 0, N / 2, 0};
  if (hipMemcpy(sd, d, sizeof(double) * N, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(sz, z, sizeof(double) * N, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(w.st, &ns, sizeof(ns), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(nd_dev, &nd, sizeof(nd), hipMemcpyHostToDevice) != hipSuccess)
    return BDC_ERR_HIP;
  launch_reset(w.ctl, w.st, w.sec, 1, st);
  launch_secular(nd_dev, 1, N, w, st);
  return finish(st);
}

int bdc_step_secular(bdc_handle_t h, int N, const double* d, const double* z, int32_t* o, double* tau,
                     int32_t* iters, bdc_stream_t stream) {
  const int rc = bdc_step_secular_start(h, N, d, z, nullptr, o, tau, iters, stream);
  return rc <= -6 && rc >= -8 ? rc + 1 : rc;  // argument positions of this signature
}

int bdc_step_gemm_ozaki(bdc_handle_t h, int slices, int M, int N, int K, const double* A, int lda,
                        const double* B, int ldb, double* C, int ldc, bdc_stream_t stream) {
  int dev, msi, mls;
  if (bdc::handle_info(h, &dev, &msi, &mls) != BDC_OK) return BDC_ERR_INVALID_HANDLE;
  if (!oz_supported(slices)) return -2;
  if (M < 0) return -3;
  if (N < 0) return -4;
  if (K < 0) return -5;
  if (M > 0 && K > 0 && !A) return -6;
  if (lda < std::max(1, M)) return -7;
  if (K > 0 && N > 0 && !B) return -8;
  if (ldb < std::max(1, K)) return -9;
  if (M > 0 && N > 0 && !C) return -10;
  if (ldc < std::max(1, M)) return -11;
  if (M == 0 || N == 0) return BDC_OK;
  Guard g(dev);
  hipStream_t st = (hipStream_t)stream;
  Tmp t;
  const int64_t P = std::max<int64_t>(32, ((int64_t)K + 31) / 32 * 32);
  unsigned short* sa = t.alloc<unsigned short>((size_t)slices * M * P);
  unsigned short* sb = t.alloc<unsigned short>((size_t)slices * N * P);
  int* ea = t.alloc<int>(M);
  int* eb = t.alloc<int>(N);
  if (!t.ok) return BDC_ERR_NOMEM;
  launch_gemm_ozaki_plain(slices, M, N, K, A, lda, B, ldb, C, ldc, sa, sb, ea, eb, P, st);
  return finish(st);
}

int bdc_step_gemm_crt(bdc_handle_t h, int moduli, int M, int N, int K, const double* A, int lda, const double* B,
                      int ldb, double* C, int ldc, bdc_stream_t stream) {
  int dev, msi, mls;
  if (bdc::handle_info(h, &dev, &msi, &mls) != BDC_OK) return BDC_ERR_INVALID_HANDLE;
  if (!crt_supported(moduli)) return -2;
  if (M < 0) return -3;
  if (N < 0) return -4;
  if (K < 0 || K > (1 << 17)) return -5;  // int32 sums exact: K * 127^2 < 2^31
  if (M > 0 && K > 0 && !A) return -6;
  if (lda < std::max(1, M)) return -7;
  if (K > 0 && N > 0 && !B) return -8;
  if (ldb < std::max(1, K)) return -9;
  if (M > 0 && N > 0 && !C) return -10;
  if (ldc < std::max(1, M)) return -11;
  if (M == 0 || N == 0) return BDC_OK;
  Guard g(dev);
  hipStream_t st = (hipStream_t)stream;
  Tmp t;
  CrtBuffers b{};
  b.base = t.alloc<char>(crt_plain_bytes(moduli, M, N, K, nullptr));
  if (!t.ok) return BDC_ERR_NOMEM;
  crt_plain_bytes(moduli, M, N, K, &b);
  launch_gemm_crt_plain(moduli, M, N, K, A, lda, B, ldb, C, ldc, b, st);
  return finish(st);
}

int bdc_step_features(bdc_handle_t h, int N, const double* d, const double* z, float* X, bdc_stream_t stream) {
  int dev, msi, mls;
  if (bdc::handle_info(h, &dev, &msi, &mls) != BDC_OK) return BDC_ERR_INVALID_HANDLE;
  if (N < 1) return -2;
  if (!d) return -3;
  if (!z) return -4;
  if (!X) return -5;
  Guard g(dev);
  hipStream_t st = (hipStream_t)stream;
  launch_features(d, z, N, X, st);
  return finish(st);
}

int bdc_step_vectors(bdc_handle_t h, int N, const double* d, const double* z, const int32_t* o,
                     const double* tau, double* zt, double* UM, double* VM, bdc_stream_t stream) {
  int dev, msi, mls;
  if (bdc::handle_info(h, &dev, &msi, &mls) != BDC_OK) return BDC_ERR_INVALID_HANDLE;
  if (N < 1) return -2;
  if (!d) return -3;
  if (!z) return -4;
  if (!o) return -5;
  if (!tau) return -6;
  if (!zt) return -7;
  if (!UM) return -8;
  if (!VM) return -9;
  Guard g(dev);
  hipStream_t st = (hipStream_t)stream;
  Tmp t;
  Work w = make_work(t, 1);
  double* sd = t.alloc<double>(N);
  double* sz = t.alloc<double>(N);
  int32_t* oo = t.alloc<int32_t>(N);
  double* tt = t.alloc<double>(N);
  int32_t* gs = t.alloc<int32_t>(N);
  NodeDesc* nd_dev = t.alloc<NodeDesc>(1);
  if (!t.ok) return BDC_ERR_NOMEM;
  w.sd = sd;
  w.sz = sz;
  w.o = oo;
  w.tau = tt;
  w.gsurv = gs;
  w.zt = zt;
  w.UM = UM;
  w.VM = VM;
  std::vector<int32_t> ident(N);
  for (int i = 0; i < N; ++i) ident[i] = i;
  NodeState ns{};
  ns.N = N;
  NodeDesc nd{0, 0, N, 0, N, 0, N / 2, 0};
  if (hipMemcpy(sd, d, sizeof(double) * N, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(sz, z, sizeof(double) * N, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(oo, o, sizeof(int32_t) * N, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(tt, tau, sizeof(double) * N, hipMemcpyDeviceToDevice) != hipSuccess ||
      hipMemcpy(gs, ident.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(w.st, &ns, sizeof(ns), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(nd_dev, &nd, sizeof(nd), hipMemcpyHostToDevice) != hipSuccess)
    return BDC_ERR_HIP;
  launch_lowner(nd_dev, 1, N, w, st);
  launch_vectors(nd_dev, 1, N, w, st);
  return finish(st);
}

int bdc_step_gemm(bdc_handle_t h, int M, int N, int K, const double* A, int lda, const double* B,
                  int ldb, double* C, int ldc, bdc_stream_t stream) {
  int dev, msi, mls;
  if (bdc::handle_info(h, &dev, &msi, &mls) != BDC_OK) return BDC_ERR_INVALID_HANDLE;
  if (M < 0) return -2;
  if (N < 0) return -3;
  if (K < 0) return -4;
  if (!A && M > 0 && K > 0) return -5;
  if (lda < std::max(1, M)) return -6;
  if (!B && K > 0 && N > 0) return -7;
  if (ldb < std::max(1, K)) return -8;
  if (!C && M > 0 && N > 0) return -9;
  if (ldc < std::max(1, M)) return -10;
  Guard g(dev);
  hipStream_t st = (hipStream_t)stream;
  launch_gemm_plain(M, N, K, A, lda, B, ldb, C, ldc, handle_tile128(h), st);
  return hipGetLastError() == hipSuccess ? BDC_OK : BDC_ERR_HIP;
}

}  // extern "C"
