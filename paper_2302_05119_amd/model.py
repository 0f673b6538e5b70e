"""Python front end of the C ABI.  PyTorch supplies device memory (the
tensors and the workspace) and the stream; all arithmetic runs in the HIP
library.  Nothing here computes any part of the method.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import Config, Stats, check, load

DTYPES = {"f64": _lib.F64, "f32": _lib.F32, "bf16": _lib.BF16, "f16": _lib.F16}


def _dbl_ptr_array(arrays):
    """Keep-alive list of contiguous float64 arrays and a C array of their pointers."""
    keep = [np.ascontiguousarray(a, dtype=np.float64) for a in arrays]
    ptrs = (ctypes.POINTER(ctypes.c_double) * len(keep))(*[a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in keep])
    return keep, ptrs


def _opt_dbl(a):
    if a is None:
        return None, None
    k = np.ascontiguousarray(a, dtype=np.float64)
    return k, k.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _void_ptr_array(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*ptrs)


def _stride_r(a, R):
    """Copy of a (rows x R^(s) or rows x R, or an R^(s)-vector) in the ABI's
    stride-R layout; the columns past R^(s) are ignored by the library."""
    a = np.asarray(a, dtype=np.float64)
    if a.shape[-1] == R:
        return a
    out = np.zeros(a.shape[:-1] + (R,), dtype=np.float64)
    out[..., :a.shape[-1]] = a
    return out


class CoupledCP:
    """Coupled nonnegative CP decomposition of S blocks of order N on one GPU.

    tensors      list of S contiguous N-way torch tensors on one HIP device
                 (float32, or float64 with compute="f64"); borrowed.  N = 3
                 has every method; N = 4..6 (the N-way model of Section II-C)
                 has the dense sweep with compute "f32" or "f64": step, fit,
                 factor(s), lam(s), lipschitz, global_fit, get/set_state,
                 debug_mttkrp and the graph_sweeps option (the others raise
                 ENOTSUP).
    rank         R; coupled = (L1, ..., LN) shared leading columns per mode
                 (default none).
    compute      "f64" | "f32" | "bf16" | "f16": MTTKRP operand type.
    init_U       optional [n][s] arrays (I_n x R); init_lambda optional [s] arrays.
    tucker_ranks optional (J1, J2, J3) or [S][3] for lra_compress.
    block_ranks  optional [S] per-block ranks R^(s) <= rank (Section II-C);
                 factors and lambdas of block s then have R^(s) columns.
    coupled_blocks optional [3] lists of the blocks that share mode n's
                 first L_n columns (None entries: every block), the flexible
                 coupling of Section III-C.
    static_workspace  True: no workspace is allocated; the context uses the
                 library's static device workspace (concpd_init_static: at
                 most one such context per device, up to
                 CONCPD_STATIC_WORKSPACE_BYTES).
    """

    def __init__(self, tensors, rank: int, coupled=None, compute: str = "f32", init_U=None, init_lambda=None,
                 seed: int = 0, update_core: bool = True, restart: bool = True, delta_w: float = 0.9999,
                 tol: float = 1e-8, max_it: int = 1000, tucker_ranks=None, block_ranks=None, coupled_blocks=None,
                 stream=None, static_workspace: bool = False):
        import torch

        self._lib = load()
        self.tensors = list(tensors)
        S = len(self.tensors)
        dev = self.tensors[0].device
        N = self.tensors[0].dim()
        for t in self.tensors:
            if t.device != dev or t.dim() != N or not t.is_contiguous():
                raise ValueError("tensors must be contiguous tensors of one order on one device")
        if not 3 <= N <= _lib.MAX_ORDER:
            raise ValueError(f"tensor order {N} not in [3, {_lib.MAX_ORDER}]")
        self.N = N
        tdt = _lib.F64 if self.tensors[0].dtype == torch.float64 else _lib.F32
        if any(t.dtype not in (torch.float32, torch.float64) or t.dtype != self.tensors[0].dtype for t in self.tensors):
            raise ValueError("tensors must all be float32 or all float64")
        self.S, self.R = S, int(rank)
        self.coupled = (0,) * N if coupled is None else tuple(int(x) for x in coupled)
        if len(self.coupled) != N:
            raise ValueError(f"coupled needs one L_n per mode ({N})")
        self.dims = [tuple(int(d) for d in t.shape) for t in self.tensors]
        self._dims_c = (ctypes.c_int64 * (N * S))(*[d for dims in self.dims for d in dims])
        self._tucker_c = None
        if tucker_ranks is not None:
            tr = np.asarray(tucker_ranks, dtype=np.int32)
            if tr.ndim == 1:
                tr = np.tile(tr, (S, 1))
            self._tucker_c = (ctypes.c_int32 * (3 * S))(*tr.reshape(-1).tolist())
        cfg = Config()
        cfg.order = N
        cfg.num_blocks = S
        cfg.rank = self.R
        for n in range(N):
            cfg.coupled[n] = self.coupled[n]
        cfg.dims = self._dims_c
        cfg.tensor_dtype = tdt
        cfg.compute_dtype = DTYPES[compute]
        cfg.update_core = int(update_core)
        cfg.restart = int(restart)
        cfg.delta_w = float(delta_w)
        cfg.tol = float(tol)
        cfg.max_it = int(max_it)
        cfg.tucker_ranks = self._tucker_c
        self.block_ranks = [self.R] * S if block_ranks is None else [int(r) for r in block_ranks]
        if len(self.block_ranks) != S:
            raise ValueError("block_ranks needs one rank per block")
        self._branks_c = (ctypes.c_int32 * S)(*self.block_ranks) if block_ranks is not None else None
        cfg.block_ranks = self._branks_c
        self._cmask_c = None
        if coupled_blocks is not None:
            masks = []
            for n in range(N):
                grp = coupled_blocks[n]
                masks.append((1 << S) - 1 if grp is None else sum(1 << int(b) for b in set(grp)))
            self._cmask_c = (ctypes.c_uint64 * N)(*masks)
        cfg.coupled_blocks = self._cmask_c
        self.cfg = cfg
        self.compute = compute
        nbytes = ctypes.c_size_t()
        check(self._lib.concpd_query_workspace(ctypes.byref(cfg), ctypes.byref(nbytes)))
        self.static_workspace = bool(static_workspace)
        if self.static_workspace:
            self.workspace = None
            self._ws_ptr = None
        else:
            self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        tptrs = _void_ptr_array([t.data_ptr() for t in self.tensors])
        keepU = keepL = None
        pU = pL = None
        if init_U is not None:
            flat = [_stride_r(init_U[n][s], self.R) for s in range(S) for n in range(N)]
            keepU, pU = _dbl_ptr_array(flat)
        if init_lambda is not None:
            keepL, pL = _dbl_ptr_array([_stride_r(x, self.R) for x in init_lambda])
        ctx = ctypes.c_void_p()
        if self.static_workspace:
            with torch.cuda.device(dev):
                check(self._lib.concpd_init_static(ctypes.byref(cfg), tptrs, pU, pL, ctypes.c_uint64(seed),
                                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        else:
            check(self._lib.concpd_init(ctypes.byref(cfg), tptrs, pU, pL, ctypes.c_uint64(seed), ctypes.c_void_p(self._ws_ptr),
                                        ctypes.c_size_t(int(nbytes.value)), ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.byref(ctx)))
        self.ctx = ctx
        del keepU, keepL

    # -- iteration --------------------------------------------------------
    def step(self, n_iter: int = 1, sync: bool = True) -> Optional[dict]:
        st = Stats()
        check(self._lib.concpd_step(self.ctx, int(n_iter), ctypes.byref(st) if sync else None))
        return st.as_dict() if sync else None

    def fit(self) -> dict:
        st = Stats()
        check(self._lib.concpd_fit(self.ctx, ctypes.byref(st)))
        return st.as_dict()

    def lra_compress(self, ranks=None) -> dict:
        st = Stats()
        pr = None
        if ranks is not None:
            r = np.asarray(ranks, dtype=np.int32)
            if r.ndim == 1:
                r = np.tile(r, (self.S, 1))
            self._ranks_c = (ctypes.c_int32 * (3 * self.S))(*r.reshape(-1).tolist())
            pr = self._ranks_c
        check(self._lib.lra_compress(self.ctx, pr, ctypes.byref(st)))
        return st.as_dict()

    def lra_compress_cp(self, init=None, eps: float = 1e-4, max_it: int = 200, seed: int = 0, rank: int = 0) -> dict:
        """Compress every block by a rank-R~ CPD fitted with ALS (the paper's own
        first step of Algorithm 2); rank R~ <= R (0: R).  init: optional [n][s]
        I_n x R~ arrays.  Returns the statistics plus 'als_iters' and
        'als_relerr' per block."""
        st = Stats()
        keep = pI = None
        if init is not None:
            keep, pI = _dbl_ptr_array([init[n][s] for s in range(self.S) for n in range(3)])
        its = (ctypes.c_int32 * self.S)()
        rel = (ctypes.c_double * self.S)()
        check(self._lib.lra_compress_cp(self.ctx, pI, ctypes.c_uint64(seed), float(eps), int(max_it), int(rank), its,
                                        rel, ctypes.byref(st)))
        del keep
        # the Kruskal form of block s has min(R~, R^(s)) columns in every mode
        rt = int(rank) or self.R
        self._ranks_c = (ctypes.c_int32 * (3 * self.S))(*[min(rt, r) for r in self.block_ranks for _ in range(3)])
        out = st.as_dict()
        out["als_iters"] = list(its)
        out["als_relerr"] = list(rel)
        return out

    def lra_step(self, n_iter: int = 1, sync: bool = True) -> Optional[dict]:
        st = Stats()
        check(self._lib.lra_step(self.ctx, int(n_iter), ctypes.byref(st) if sync else None))
        return st.as_dict() if sync else None

    def tucker(self, s: int):
        """Compressed form of block s after lra_compress: ([A_1, A_2, A_3], G)."""
        P = ctypes.POINTER(ctypes.c_double)
        J = self._tucker_ranks(s)
        A = []
        for n in range(3):
            a = np.empty((self.dims[s][n], J[n]), dtype=np.float64)
            check(self._lib.lra_get_tucker(self.ctx, s, n, a.ctypes.data_as(P)))
            A.append(a)
        G = np.empty(tuple(J), dtype=np.float64)
        check(self._lib.lra_get_tucker(self.ctx, s, 3, G.ctypes.data_as(P)))
        return A, G

    def _tucker_ranks(self, s: int):
        src = getattr(self, "_ranks_c", None) or self._tucker_c
        return [int(src[3 * s + n]) for n in range(3)]

    def loss_grad(self, U, lam, coupled: bool = False):
        """F and its gradients at the point (U [n][s] device tensors I_n x R in the
        factor type, lam [s] device float64 R-vectors).  Returns (F, gU [n][s],
        glam [s]); with coupled=True the shared columns come from block 0 and
        every block receives the gradient with respect to them (summed over s)."""
        import torch

        ftype = torch.float64 if self.compute == "f64" else torch.float32
        dev = self.tensors[0].device
        Uc = [[None] * self.S for _ in range(3)]
        for n in range(3):
            for s in range(self.S):
                t = U[n][s]
                if t.dtype != ftype or t.device != dev or tuple(t.shape) != (self.dims[s][n], self.R):
                    raise ValueError(f"U[{n}][{s}] must be a {ftype} tensor of shape {(self.dims[s][n], self.R)} on {dev}")
                Uc[n][s] = t.contiguous()
        lc = []
        for s in range(self.S):
            t = lam[s]
            if t.dtype != torch.float64 or t.device != dev or t.numel() != self.R:
                raise ValueError(f"lam[{s}] must be a float64 tensor of {self.R} entries on {dev}")
            lc.append(t.contiguous())
        gU = [[torch.empty_like(Uc[n][s]) for s in range(self.S)] for n in range(3)]
        gl = [torch.empty_like(lc[s]) for s in range(self.S)]
        order = [(n, s) for s in range(self.S) for n in range(3)]
        pU = _void_ptr_array([Uc[n][s].data_ptr() for n, s in order])
        pL = _void_ptr_array([t.data_ptr() for t in lc])
        pgU = _void_ptr_array([gU[n][s].data_ptr() for n, s in order])
        pgL = _void_ptr_array([t.data_ptr() for t in gl])
        F = ctypes.c_double()
        torch.cuda.current_stream(dev).synchronize()
        check(self._lib.concpd_loss_grad(self.ctx, pU, pL, int(bool(coupled)), ctypes.byref(F), pgU, pgL))
        return F.value, gU, gl

    # -- launch options (batching form) -------------------------------------
    _OPTS = {"graph_sweeps": _lib.OPT_GRAPH_SWEEPS, "overlap": _lib.OPT_OVERLAP, "k2_rows": _lib.OPT_K2_ROWS,
             "p1_split": _lib.OPT_P1_SPLIT, "p1_dma": _lib.OPT_P1_DMA, "fuse": _lib.OPT_FUSE,
             "fuse_lra": _lib.OPT_FUSE_LRA}

    def set_option(self, name: str, value: int) -> None:
        check(self._lib.concpd_set_option(self.ctx, self._OPTS[name], int(value)))

    def get_option(self, name: str) -> int:
        v = ctypes.c_int64()
        check(self._lib.concpd_get_option(self.ctx, self._OPTS[name], ctypes.byref(v)))
        return v.value

    def autotune(self, sweeps: int = 20) -> dict:
        t = _lib.Tuning()
        check(self._lib.concpd_autotune(self.ctx, int(sweeps), ctypes.byref(t)))
        return t.as_dict()

    def stats(self) -> dict:
        return self.step(0)

    # -- read-back --------------------------------------------------------
    def factor(self, n: int, s: int, padded: bool = False) -> np.ndarray:
        """U^(n,s), I_n x R^(s) (I_n x R with the zero columns if padded)."""
        out = np.empty((self.dims[s][n], self.R), dtype=np.float64)
        check(self._lib.concpd_get_factor(self.ctx, n, s, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out if padded else out[:, :self.block_ranks[s]].copy()

    def factors(self):
        return [[self.factor(n, s) for s in range(self.S)] for n in range(self.N)]

    def lam(self, s: int, padded: bool = False) -> np.ndarray:
        out = np.empty(self.R, dtype=np.float64)
        check(self._lib.concpd_get_lambda(self.ctx, s, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out if padded else out[:self.block_ranks[s]].copy()

    def lams(self):
        return [self.lam(s) for s in range(self.S)]

    def lipschitz(self):
        Ld = np.empty(self.S)
        Lu = np.empty(self.N * self.S)
        LC = np.empty(self.N)
        P = ctypes.POINTER(ctypes.c_double)
        check(self._lib.concpd_get_lipschitz(self.ctx, Ld.ctypes.data_as(P), Lu.ctypes.data_as(P), LC.ctypes.data_as(P)))
        return Ld, Lu.reshape(self.S, self.N), LC

    def global_fit(self) -> float:
        f = ctypes.c_double()
        check(self._lib.concpd_global_fit(self.ctx, ctypes.byref(f)))
        return f.value

    def debug_mttkrp(self, n: int, s: int):
        import torch

        dt = torch.float64 if self.compute == "f64" else torch.float32
        out = torch.empty((self.dims[s][n], self.R), dtype=dt, device=self.tensors[0].device)
        check(self._lib.concpd_debug_mttkrp(self.ctx, n, s, ctypes.c_void_p(out.data_ptr())))
        return out

    def get_state(self) -> dict:
        """The iterate state for a checkpoint, as keyword arguments of
        set_state: U, U_prev [n][s] (I_n x R^(s)), lam, lam_prev [s],
        Ld_prev [s], Lu_prev [s][n], LC_prev [n] (None where unset), t, k."""
        S, N = self.S, self.N
        bufs = {key: [[np.zeros((self.dims[s][n], self.R)) for s in range(S)] for n in range(N)] for key in ("U", "U_prev")}
        lams = {key: [np.zeros(self.R) for _ in range(S)] for key in ("lam", "lam_prev")}
        P = ctypes.POINTER(ctypes.c_double)
        flat = lambda UU: (P * (N * S))(*[UU[n][s].ctypes.data_as(P) for s in range(S) for n in range(N)])  # noqa: E731
        lptr = lambda LL: (P * S)(*[x.ctypes.data_as(P) for x in LL])  # noqa: E731
        Ld, Lu, LC = np.zeros(S), np.zeros(N * S), np.zeros(N)
        t = ctypes.c_double()
        k = ctypes.c_int64()
        check(self._lib.concpd_get_state(self.ctx, flat(bufs["U"]), flat(bufs["U_prev"]), lptr(lams["lam"]),
                                         lptr(lams["lam_prev"]), Ld.ctypes.data_as(P), Lu.ctypes.data_as(P),
                                         LC.ctypes.data_as(P), ctypes.byref(t), ctypes.byref(k)))
        r = self.block_ranks
        none = lambda v: None if v < 0 else float(v)  # noqa: E731
        return {"U": [[bufs["U"][n][s][:, :r[s]] for s in range(S)] for n in range(N)],
                "U_prev": [[bufs["U_prev"][n][s][:, :r[s]] for s in range(S)] for n in range(N)],
                "lam": [lams["lam"][s][:r[s]] for s in range(S)], "lam_prev": [lams["lam_prev"][s][:r[s]] for s in range(S)],
                "Ld_prev": [none(v) for v in Ld], "Lu_prev": [[none(v) for v in Lu[N * s:N * s + N]] for s in range(S)],
                "LC_prev": [none(v) for v in LC], "t": t.value, "k": k.value}

    def set_state(self, U, lam, U_prev=None, lam_prev=None, Ld_prev=None, Lu_prev=None, LC_prev=None, t=1.0, k=0):
        """U, U_prev: [n][s] arrays; Lu_prev [s][n] (or [n][s] transposed by caller); None entries mean 'none'."""
        flat = lambda UU: [_stride_r(UU[n][s], self.R) for s in range(self.S) for n in range(self.N)]  # noqa: E731
        kU, pU = _dbl_ptr_array(flat(U))
        kL, pL = _dbl_ptr_array([_stride_r(x, self.R) for x in lam])
        kUp = pUp = kLp = pLp = None
        if U_prev is not None:
            kUp, pUp = _dbl_ptr_array(flat(U_prev))
        if lam_prev is not None:
            kLp, pLp = _dbl_ptr_array([_stride_r(x, self.R) for x in lam_prev])

        def _arr(x, shape):
            if x is None:
                return None, None
            a = np.array([(-1.0 if v is None else float(v)) for v in np.asarray(x, dtype=object).reshape(-1)],
                         dtype=np.float64).reshape(shape)
            return _opt_dbl(a)

        kd, pd = _arr(Ld_prev, (self.S,))
        ku, pu = _arr(Lu_prev, (self.S, self.N))
        kc, pc = _arr(LC_prev, (self.N,))
        check(self._lib.concpd_set_state(self.ctx, pU, pUp, pL, pLp, pd, pu, pc, float(t), int(k)))
        del kU, kL, kUp, kLp, kd, ku, kc

    def profile(self, enable: bool = True):
        check(self._lib.concpd_profile(self.ctx, int(enable)))

    def profile_read(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_int64()
        check(self._lib.concpd_profile_read(self.ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)))
        return a.value, b.value, n.value

    def close(self):
        if getattr(self, "ctx", None):
            check(self._lib.concpd_destroy(self.ctx))
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def launch_floor(kernels: int, reps: int = 2000) -> dict:
    """Launch-latency floor of a sweep of `kernels` kernels: microseconds per
    replay of a graph of that many empty kernels, and per as many direct
    launches (device-side HIP events)."""
    lib = load()
    g, d = ctypes.c_double(), ctypes.c_double()
    check(lib.concpd_launch_floor(int(kernels), int(reps), ctypes.byref(g), ctypes.byref(d)))
    return {"kernels": int(kernels), "graph_us": g.value, "direct_us": d.value}


def spectral_norm(mats) -> np.ndarray:
    """Largest eigenvalues of symmetric n x n FP64 matrices ([count, n, n] or
    [n, n]) computed on the device by the sweep's spectral-norm code (the
    Lipschitz constants of eqs. eqLipsLd / eqLipsLu)."""
    a = np.ascontiguousarray(np.asarray(mats, dtype=np.float64))
    single = a.ndim == 2
    if single:
        a = a[None]
    if a.ndim != 3 or a.shape[1] != a.shape[2]:
        raise ValueError("expected [count, n, n] or [n, n]")
    out = np.zeros(a.shape[0], dtype=np.float64)
    lib = load()
    check(lib.concpd_debug_spectral_norm(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.shape[1], a.shape[0],
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out[0] if single else out
