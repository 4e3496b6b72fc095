"""Python binding of the bidiagonal divide-and-conquer SVD (torch tensors in,
torch tensors out).  Argument marshalling only: every step of the solve runs
in the HIP kernels of libbdc.so, which must be built; there is no fallback.
"""

from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _f64(t, device) -> torch.Tensor:
    t = torch.as_tensor(t, dtype=torch.float64, device=device)
    return t.contiguous()


class Solver:
    """One handle of the C ABI (workspace, plan cache) on one GPU."""

    def __init__(self, device: int | torch.device = 0, leaf_size: int = 32, max_secular_iters: int = 64,
                 max_leaf_sweeps: int = 40, workspace_cap_bytes: int = 0, timing: bool = False,
                 use_graph: bool = True, start: str = "plain", mlp_params=None, gemm: str = "fp64",
                 ozaki_slices: int = 7, ozaki_min_n: int = 256, crt_moduli: int = 16,
                 learned_min_n: int | None = None):
        """start: "plain" (midpoint) or "learned" (the MLP's proposal; the
        parameters come from ``mlp_params`` (host float32 vector) or, when
        that is None, from the network file shipped with the package), for
        merges of at least ``learned_min_n`` kept values (None: the library's
        default; 0: every merge).
        gemm: "fp64", "ozaki" (bfloat16-slice split products) or "crt" (int8
        residue split products with ``crt_moduli`` moduli), the split forms
        for merges with at least ``ozaki_min_n`` kept values in
        single-problem solves."""
        self.lib = _lib.load()
        dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if dev.type != "cuda":
            raise ValueError("the solver runs on a GPU device")
        self.device = torch.device("cuda", dev.index if dev.index is not None else 0)
        opt = _lib.Options()
        self.lib.bdc_default_options(ctypes.byref(opt))
        opt.leaf_size = leaf_size
        opt.max_secular_iters = max_secular_iters
        opt.max_leaf_sweeps = max_leaf_sweeps
        opt.workspace_cap_bytes = workspace_cap_bytes
        opt.timing = 1 if timing else 0
        opt.use_graph = 1 if use_graph else 0
        if start not in ("plain", "learned"):
            raise ValueError("start must be 'plain' or 'learned'")
        opt.start = _lib.BDC_START_LEARNED if start == "learned" else _lib.BDC_START_PLAIN
        gemms = {"fp64": _lib.BDC_GEMM_FP64, "ozaki": _lib.BDC_GEMM_OZAKI, "crt": _lib.BDC_GEMM_CRT}
        if gemm not in gemms:
            raise ValueError("gemm must be 'fp64', 'ozaki' or 'crt'")
        opt.gemm = gemms[gemm]
        opt.ozaki_slices = ozaki_slices
        opt.ozaki_min_n = ozaki_min_n
        opt.crt_moduli = crt_moduli
        if learned_min_n is not None:
            opt.learned_min_n = learned_min_n
        self.options = opt
        h = ctypes.c_void_p()
        check("bdc_create", self.lib.bdc_create(ctypes.byref(h), self.device.index, ctypes.byref(opt)))
        self.handle = h
        if mlp_params is None and start == "learned":
            from .start_model import load_params
            mlp_params = load_params()
        if mlp_params is not None:
            self.mlp_set(mlp_params)

    def close(self) -> None:
        if self.handle:
            self.lib.bdc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self) -> int:
        return torch.cuda.current_stream(self.device).cuda_stream

    # ---------------------------------------------------------------- solves
    def svd(self, d, e, out=None):
        """B = U diag(sigma) VT for the n x n upper bidiagonal (d, e).

        Returns (sigma, U, VT) as float64 tensors on the device; sigma is
        descending.  ``out`` may supply (sigma, Ubuf, VTbuf) buffers of shapes
        (n,), (n, n), (n, n); U and VT are returned as transposed views of the
        column-major buffers."""
        d = _f64(d, self.device)
        n = d.shape[0]
        e = _f64(e, self.device) if n > 1 else None
        if e is not None and e.shape[0] < n - 1:
            raise ValueError("e must hold n-1 entries")
        if out is None:
            sigma = torch.empty(n, dtype=torch.float64, device=self.device)
            ub = torch.empty((n, n), dtype=torch.float64, device=self.device)
            vb = torch.empty((n, n), dtype=torch.float64, device=self.device)
        else:
            sigma, ub, vb = out
        check("bdc_svd", self.lib.bdc_svd(self.handle, n, _ptr(d), _ptr(e), _ptr(sigma), _ptr(ub),
                                          _ptr(vb), self._stream()))
        return sigma, ub.T, vb.T

    def svd_batched(self, sizes, d, e, out=None):
        """Many bidiagonals in one call.  d, e packed at offsets sum(n_j);
        returns (sigma packed like d, U packed, VT packed), where problem i's
        U is ``U[mo_i : mo_i + n_i*n_i].view(n_i, n_i).T`` with
        mo_i = sum_{j<i} n_j^2 (column-major storage)."""
        sizes = [int(x) for x in sizes]
        arr = (ctypes.c_int64 * max(1, len(sizes)))(*sizes)
        d = _f64(d, self.device)
        e = _f64(e, self.device)
        tot = sum(sizes)
        tot2 = sum(x * x for x in sizes)
        if out is None:
            sigma = torch.empty(tot, dtype=torch.float64, device=self.device)
            U = torch.empty(tot2, dtype=torch.float64, device=self.device)
            VT = torch.empty(tot2, dtype=torch.float64, device=self.device)
        else:
            sigma, U, VT = out
        check("bdc_svd_batched", self.lib.bdc_svd_batched(self.handle, len(sizes), arr, _ptr(d), _ptr(e),
                                                          _ptr(sigma), _ptr(U), _ptr(VT), self._stream()))
        return sigma, U, VT

    def info(self):
        """(info, stats dict) of the last solve (synchronises)."""
        info = ctypes.c_int64()
        st = _lib.Stats()
        check("bdc_get_info", self.lib.bdc_get_info(self.handle, ctypes.byref(info), ctypes.byref(st)))
        return int(info.value), st.as_dict()

    def timing(self) -> dict:
        cap = 32
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_int64 * cap)()
        k = self.lib.bdc_get_timing(self.handle, cap, names, ms, cnt)
        if k < 0:
            raise _lib.BdcError("bdc_get_timing", k)
        return {names[i].decode(): (ms[i], int(cnt[i])) for i in range(k)}

    def clear_timing(self) -> None:
        check("bdc_clear_timing", self.lib.bdc_clear_timing(self.handle))

    # ---------------------------------------------------------------- tuning
    def tuning(self) -> dict:
        t = _lib.Tuning()
        check("bdc_get_tuning", self.lib.bdc_get_tuning(self.handle, ctypes.byref(t)))
        d = t.as_dict()
        d.pop("ms")
        return d

    def set_tuning(self, small_n: int, flat: int, grid64: int, grid128: int, sec_small_n: int = 256,
                   leaf_size: int = 0, tile128: int = 1, streams: int = 1, **_ignored) -> None:
        t = _lib.Tuning(small_n, flat, grid64, grid128, sec_small_n, leaf_size, tile128, streams, 0.0)
        check("bdc_set_tuning", self.lib.bdc_set_tuning(self.handle, ctypes.byref(t)))

    def autotune(self, sizes, d, e, out=None, repeats: int = 2) -> dict:
        """Time the candidate launch tunings on this workload (a batch given by
        ``sizes`` with packed d, e) and keep the fastest; returns it."""
        sizes = [int(x) for x in sizes]
        arr = (ctypes.c_int64 * max(1, len(sizes)))(*sizes)
        d = _f64(d, self.device)
        e = _f64(e, self.device)
        tot = sum(sizes)
        tot2 = sum(x * x for x in sizes)
        if out is None:
            out = (torch.empty(tot, dtype=torch.float64, device=self.device),
                   torch.empty(tot2, dtype=torch.float64, device=self.device),
                   torch.empty(tot2, dtype=torch.float64, device=self.device))
        best = _lib.Tuning()
        check("bdc_autotune", self.lib.bdc_autotune(self.handle, len(sizes), arr, _ptr(d), _ptr(e), _ptr(out[0]),
                                                    _ptr(out[1]), _ptr(out[2]), self._stream(), repeats,
                                                    ctypes.byref(best)))
        return best.as_dict()

    # ---------------------------------------------------------------- learned start
    def mlp_set(self, params) -> None:
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if p.shape != (_lib.MLP_PARAMS,):
            raise ValueError(f"expected {_lib.MLP_PARAMS} parameters")
        check("bdc_mlp_set", self.lib.bdc_mlp_set(self.handle, p.ctypes.data, p.shape[0]))

    def mlp_get(self):
        import numpy as np
        p = np.empty(_lib.MLP_PARAMS, dtype=np.float32)
        check("bdc_mlp_get", self.lib.bdc_mlp_get(self.handle, p.ctypes.data, p.shape[0]))
        return p

    def mlp_forward(self, X: torch.Tensor) -> torch.Tensor:
        X = torch.as_tensor(X, dtype=torch.float32, device=self.device).contiguous()
        rows = X.shape[0]
        out = torch.empty(rows, dtype=torch.float32, device=self.device)
        check("bdc_mlp_forward", self.lib.bdc_mlp_forward(self.handle, _ptr(X), rows, _ptr(out), self._stream()))
        return out

    def mlp_grad(self, X, y):
        X = torch.as_tensor(X, dtype=torch.float32, device=self.device).contiguous()
        y = torch.as_tensor(y, dtype=torch.float32, device=self.device).contiguous()
        g = torch.empty(_lib.MLP_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        check("bdc_mlp_grad", self.lib.bdc_mlp_grad(self.handle, _ptr(X), _ptr(y), X.shape[0], _ptr(g), _ptr(loss),
                                                    self._stream()))
        return float(loss.item()), g

    def mlp_train(self, X: torch.Tensor, y: torch.Tensor, idx: torch.Tensor, batch: int, lr: float):
        """len(idx) // batch Adam steps over rows idx (device int32);
        returns the per-step batch losses (device tensor)."""
        steps = idx.shape[0] // batch
        hist = torch.empty(max(steps, 1), dtype=torch.float32, device=self.device)
        check("bdc_mlp_train", self.lib.bdc_mlp_train(self.handle, _ptr(X), _ptr(y), _ptr(idx), batch, steps,
                                                      float(lr), _ptr(hist), self._stream()))
        return hist[:steps]

    def harvest(self, capacity: int):
        """Start collecting training rows from later solves; returns
        (X, y, tag, count) device buffers (count: rows seen so far)."""
        X = torch.empty((capacity, _lib.MLP_FEATURES), dtype=torch.float32, device=self.device)
        y = torch.empty(capacity, dtype=torch.float32, device=self.device)
        tag = torch.empty((capacity, 3), dtype=torch.int32, device=self.device)
        count = torch.zeros(1, dtype=torch.int64, device=self.device)
        check("bdc_set_harvest", self.lib.bdc_set_harvest(self.handle, _ptr(X), _ptr(y), _ptr(tag), capacity,
                                                          _ptr(count)))
        self._harvest = (X, y, tag, count)
        return self._harvest

    def stop_harvest(self) -> None:
        check("bdc_set_harvest", self.lib.bdc_set_harvest(self.handle, None, None, None, 0, None))
        self._harvest = None

    # ---------------------------------------------------------------- back-transformation
    def apply_reflectors(self, Y: torch.Tensor, tau: torch.Tensor, C: torch.Tensor, trans: bool = False,
                         offset: int = 0, rows: bool = False, block: int = 0, noalloc: bool = False) -> torch.Tensor:
        """C <- Q C (or Q^T C) in place for Q = H_0 ... H_{k-1}: reflector i
        in column i of Y (rows=False; Y is (m, k)) or row i (rows=True; Y is
        (k, m)), unit pivot at i + offset, stored entries below it.  C is a
        (m, p) float64 tensor whose memory is column-major (pass the .T of a
        contiguous (p, m) tensor).  noalloc=True calls the allocation-free
        entry point (fixed per-GPU scratch; same results)."""
        m, p = C.shape
        # strides of size-1 dimensions carry no layout (torch sets them freely)
        ldc = C.stride(1) if p > 1 else max(1, m)
        if (m > 1 and C.stride(0) != 1) or ldc < max(1, m):
            raise ValueError("C must be column-major (the transpose of a contiguous tensor)")
        k = tau.shape[0]
        if rows:
            rs, cs = Y.stride(1), Y.stride(0)
        else:
            rs, cs = Y.stride(0), Y.stride(1)
        name = "bdc_apply_reflectors_noalloc" if noalloc else "bdc_apply_reflectors"
        check(name, getattr(self.lib, name)(
            self.handle, 1 if trans else 0, m, p, k, offset, _ptr(Y), rs, cs, _ptr(tau), _ptr(C), ldc,
            block, self._stream()))
        return C

    # ---------------------------------------------------------------- tall-and-skinny QR
    @staticmethod
    def _colmajor_ld(X: torch.Tensor, name: str) -> int:
        """Leading dimension of a (rows, cols) float64 view of column-major
        memory (the .T of a contiguous (cols, rows) tensor)."""
        r, c = X.shape
        ld = X.stride(1) if c > 1 else max(1, r)
        if X.dtype != torch.float64 or (r > 1 and X.stride(0) != 1) or ld < max(1, r):
            raise ValueError(f"{name} must be float64 and column-major (the transpose of a contiguous tensor)")
        return ld

    def gebrd(self, A: torch.Tensor, block: int = 0):
        """A (m, n), m >= n, column-major float64 on the device, is overwritten
        with the bidiagonal and the reflectors (LAPACK's gebrd storage);
        returns (d, e, tauq, taup)."""
        m, n = A.shape
        lda = self._colmajor_ld(A, "A")
        d = torch.empty(n, dtype=torch.float64, device=self.device)
        e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=self.device)
        tq = torch.empty(n, dtype=torch.float64, device=self.device)
        tp = torch.empty(n, dtype=torch.float64, device=self.device)
        check("bdc_gebrd", self.lib.bdc_gebrd(self.handle, m, n, _ptr(A), lda, _ptr(d), _ptr(e), _ptr(tq), _ptr(tp),
                                              block, self._stream()))
        return d, e[:max(n - 1, 0)], tq, tp

    def geqrf(self, A: torch.Tensor, block: int = 0) -> torch.Tensor:
        """A (m, n), m >= n, column-major float64 on the device, is overwritten
        with R and the Householder vectors (LAPACK's geqrf storage); returns
        tau (n)."""
        m, n = A.shape
        lda = self._colmajor_ld(A, "A")
        tau = torch.empty(n, dtype=torch.float64, device=self.device)
        check("bdc_geqrf", self.lib.bdc_geqrf(self.handle, m, n, _ptr(A), lda, _ptr(tau), block, self._stream()))
        return tau

    def orgqr(self, A: torch.Tensor, tau: torch.Tensor, ncols: int | None = None, block: int = 0) -> torch.Tensor:
        """The first ncols (default n) columns of Q = H_0 ... H_{n-1} from
        geqrf's A and tau, as an (m, ncols) column-major tensor."""
        m, n = A.shape
        lda = self._colmajor_ld(A, "A")
        nc = n if ncols is None else int(ncols)
        k = tau.shape[0]
        Q = torch.empty((nc, m), dtype=torch.float64, device=self.device).T
        check("bdc_orgqr", self.lib.bdc_orgqr(self.handle, m, nc, k, _ptr(A), lda, _ptr(tau), _ptr(Q), max(1, m),
                                              block, self._stream()))
        return Q

    # ---------------------------------------------------------------- steps
    def step_leaf(self, d, e, s: int):
        d = _f64(d, self.device)
        m = d.shape[0]
        e = _f64(e, self.device) if m - 1 + s > 0 else None
        sig = torch.empty(m, dtype=torch.float64, device=self.device)
        W = torch.empty((m, m), dtype=torch.float64, device=self.device)
        Q = torch.empty((m + s, m + s), dtype=torch.float64, device=self.device)
        check("bdc_step_leaf", self.lib.bdc_step_leaf(self.handle, m, s, _ptr(d), _ptr(e), _ptr(sig), _ptr(W),
                                                      _ptr(Q), self._stream()))
        return sig, W.T, Q.T

    def step_deflate(self, m: int, s: int, sig, qrow1, qrow2, alpha: float, beta: float) -> dict:
        sig = _f64(sig, self.device)
        q1 = _f64(qrow1, self.device)
        q2 = _f64(qrow2, self.device)
        dev = self.device
        perm = torch.empty(m, dtype=torch.int32, device=dev)
        dz = torch.empty(2 * m, dtype=torch.float64, device=dev)
        status = torch.empty(m, dtype=torch.int32, device=dev)
        rot_pos = torch.zeros(2 * m, dtype=torch.int32, device=dev)
        rot_cs = torch.zeros(2 * m, dtype=torch.float64, device=dev)
        misc = torch.empty(8, dtype=torch.float64, device=dev)
        nrot = torch.zeros(1, dtype=torch.int32, device=dev)
        check("bdc_step_deflate", self.lib.bdc_step_deflate(
            self.handle, m, s, _ptr(sig), _ptr(q1), _ptr(q2), float(alpha), float(beta), _ptr(perm), _ptr(dz),
            _ptr(status), _ptr(rot_pos), _ptr(rot_cs), _ptr(misc), _ptr(nrot), self._stream()))
        nr = int(nrot.item())
        misc = misc.cpu().numpy()
        return {
            "perm": perm.cpu().numpy(), "d": dz[:m].cpu().numpy(), "z": dz[m:].cpu().numpy(),
            "status": status.cpu().numpy(), "rot_pos": rot_pos[: 2 * nr].cpu().numpy().reshape(-1, 2),
            "rot_cs": rot_cs[: 2 * nr].cpu().numpy().reshape(-1, 2), "scale": misc[0], "tol": misc[1],
            "c0": misc[2], "s0": misc[3], "N": int(misc[4]), "counts": (int(misc[5]), int(misc[6]), int(misc[7])),
        }

    def step_secular(self, d, z):
        d = _f64(d, self.device)
        z = _f64(z, self.device)
        N = d.shape[0]
        o = torch.empty(N, dtype=torch.int32, device=self.device)
        tau = torch.empty(N, dtype=torch.float64, device=self.device)
        it = torch.empty(N, dtype=torch.int32, device=self.device)
        check("bdc_step_secular", self.lib.bdc_step_secular(self.handle, N, _ptr(d), _ptr(z), _ptr(o), _ptr(tau),
                                                            _ptr(it), self._stream()))
        return o, tau, it

    def step_secular_start(self, d, z, xstart):
        d = _f64(d, self.device)
        z = _f64(z, self.device)
        xs = torch.as_tensor(xstart, dtype=torch.float32, device=self.device).contiguous()
        N = d.shape[0]
        o = torch.empty(N, dtype=torch.int32, device=self.device)
        tau = torch.empty(N, dtype=torch.float64, device=self.device)
        it = torch.empty(N, dtype=torch.int32, device=self.device)
        check("bdc_step_secular_start", self.lib.bdc_step_secular_start(
            self.handle, N, _ptr(d), _ptr(z), _ptr(xs), _ptr(o), _ptr(tau), _ptr(it), self._stream()))
        return o, tau, it

    def step_features(self, d, z):
        d = _f64(d, self.device)
        z = _f64(z, self.device)
        N = d.shape[0]
        X = torch.empty((N, _lib.MLP_FEATURES), dtype=torch.float32, device=self.device)
        check("bdc_step_features", self.lib.bdc_step_features(self.handle, N, _ptr(d), _ptr(z), _ptr(X),
                                                              self._stream()))
        return X

    def step_vectors(self, d, z, o, tau):
        d = _f64(d, self.device)
        z = _f64(z, self.device)
        o = torch.as_tensor(o, dtype=torch.int32, device=self.device).contiguous()
        tau = _f64(tau, self.device)
        N = d.shape[0]
        zt = torch.empty(N, dtype=torch.float64, device=self.device)
        UM = torch.empty((N, N), dtype=torch.float64, device=self.device)
        VM = torch.empty((N, N), dtype=torch.float64, device=self.device)
        check("bdc_step_vectors", self.lib.bdc_step_vectors(self.handle, N, _ptr(d), _ptr(z), _ptr(o), _ptr(tau),
                                                            _ptr(zt), _ptr(UM), _ptr(VM), self._stream()))
        return zt, UM.T, VM.T

    def gemm(self, A: torch.Tensor, B: torch.Tensor, C: torch.Tensor) -> None:
        """C (M, N) = A (M, K) @ B (K, N) on column-major float64 device views
        (bdc_step_gemm, the FP64 matrix-core kernel; no copies)."""
        M, K = A.shape
        K2, N = B.shape
        if K != K2 or tuple(C.shape) != (M, N):
            raise ValueError("gemm: shapes do not match")
        lda, ldb, ldc = self._colmajor_ld(A, "A"), self._colmajor_ld(B, "B"), self._colmajor_ld(C, "C")
        check("bdc_step_gemm", self.lib.bdc_step_gemm(self.handle, M, N, K, _ptr(A), lda, _ptr(B), ldb, _ptr(C), ldc,
                                                      self._stream()))

    def step_gemm(self, A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
        """C = A @ B through the update kernel (A, B float64 on the device)."""
        M, K = A.shape
        K2, N = B.shape
        assert K == K2
        Ac = A.T.contiguous()  # column-major storage
        Bc = B.T.contiguous()
        C = torch.empty((N, M), dtype=torch.float64, device=self.device)
        check("bdc_step_gemm", self.lib.bdc_step_gemm(self.handle, M, N, K, _ptr(Ac), max(1, M), _ptr(Bc),
                                                      max(1, K), _ptr(C), max(1, M), self._stream()))
        return C.T

    def step_gemm_ozaki(self, A: torch.Tensor, B: torch.Tensor, slices: int = 7) -> torch.Tensor:
        """C = A @ B through the split-precision kernels."""
        M, K = A.shape
        K2, N = B.shape
        assert K == K2
        Ac = A.T.contiguous()
        Bc = B.T.contiguous()
        C = torch.empty((N, M), dtype=torch.float64, device=self.device)
        check("bdc_step_gemm_ozaki", self.lib.bdc_step_gemm_ozaki(
            self.handle, slices, M, N, K, _ptr(Ac), max(1, M), _ptr(Bc), max(1, K), _ptr(C), max(1, M),
            self._stream()))
        return C.T


    def step_gemm_crt(self, A: torch.Tensor, B: torch.Tensor, moduli: int = 16) -> torch.Tensor:
        """C = A @ B through the int8 residue (Chinese remainder) kernels."""
        M, K = A.shape
        K2, N = B.shape
        assert K == K2
        Ac = A.T.contiguous()
        Bc = B.T.contiguous()
        C = torch.empty((N, M), dtype=torch.float64, device=self.device)
        check("bdc_step_gemm_crt", self.lib.bdc_step_gemm_crt(
            self.handle, moduli, M, N, K, _ptr(Ac), max(1, M), _ptr(Bc), max(1, K), _ptr(C), max(1, M),
            self._stream()))
        return C.T

_DEFAULT: dict = {}


def svd(d, e, device: int = 0):
    """B = U diag(sigma) VT on the GPU with a cached default solver."""
    s = _DEFAULT.get(device)
    if s is None:
        s = _DEFAULT[device] = Solver(device)
    return s.svd(d, e)
