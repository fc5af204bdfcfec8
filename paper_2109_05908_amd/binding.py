"""ctypes binding of libdd.so: argument marshalling only.

Every function here forwards to the C-ABI of include/dd.h with raw device
pointers taken from torch tensors and the current HIP stream.  No arithmetic
of the method happens in Python.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

DD_FP64, DD_FP32 = 0, 1
DD_SEL_THRESHOLD, DD_SEL_THRESHOLD_CAP = 0, 1
DD_SCHWARZ_ADDITIVE, DD_SCHWARZ_DEFLATED = 0, 1
DD_EIG_DENSE, DD_EIG_LOBPCG, DD_EIG_LOBPCG_MATFREE = 0, 1, 2
DD_START_RANDOM, DD_START_RANGE, DD_START_MODEL = 0, 1, 2
DD_ERR_INVALID_ARG, DD_ERR_NOT_SPD, DD_ERR_EIG, DD_ERR_NAN, DD_ERR_OOM, DD_ERR_HIP = -1, -2, -3, -4, -5, -6
DD_NPHASE = 12
DD_MAX_LEVELS = 4
DD_PHIST = 16


class DDError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = lib().dd_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{what}: {msg} (code {code})")


class _Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p), ("colind", C.c_void_p),
                ("val", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("local_prec", C.c_int32), ("select", C.c_int32), ("nev_cap", C.c_int32),
                ("validate", C.c_int32), ("coarsen", C.c_int32), ("schwarz", C.c_int32),
                ("eig_solver", C.c_int32), ("lobpcg_maxit", C.c_int32), ("lobpcg_tol", C.c_double),
                ("warm_start", C.c_int32), ("graph_pcg", C.c_int32), ("seed", C.c_uint64),
                ("warm_start_model", C.c_void_p), ("reserved", C.c_int32 * 8)]


def _opts(local_prec=0, select=0, nev_cap=0, validate=False, coarsen=0, schwarz=0, eig_solver=0, lobpcg_maxit=0,
          lobpcg_tol=0.0, warm_start=0, seed=0, model=None, graph_pcg=0):
    o = _Opts()
    o.local_prec, o.select, o.nev_cap, o.validate = local_prec, select, nev_cap, int(validate)
    o.coarsen, o.schwarz, o.eig_solver, o.lobpcg_maxit = int(coarsen), int(schwarz), int(eig_solver), int(lobpcg_maxit)
    o.lobpcg_tol, o.warm_start, o.seed = float(lobpcg_tol), int(warm_start), int(seed)
    o.graph_pcg = int(graph_pcg)
    o.warm_start_model = model._h if model is not None else None
    return o


class _Info(C.Structure):
    _fields_ = [("levels", C.c_int32), ("N", C.c_int32 * DD_MAX_LEVELS), ("n", C.c_int64 * DD_MAX_LEVELS),
                ("n_C", C.c_int64), ("grid_complexity", C.c_double), ("p_min", C.c_int32),
                ("p_max", C.c_int32), ("p_hist", C.c_int32 * DD_PHIST), ("k_c", C.c_int32),
                ("fp32_fallbacks", C.c_int32), ("eig_maxit_hits", C.c_int32), ("eig_iters_max", C.c_int32),
                ("eig_iters_mean", C.c_double), ("eig_resid_max", C.c_double),
                ("phase_ms", C.c_double * DD_NPHASE), ("last_iters", C.c_int32), ("last_relres", C.c_double),
                ("device_bytes", C.c_int64), ("coarse_factor_bytes", C.c_int64)]


class _Meter(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("flops", C.c_double), ("bytes", C.c_double)]


def meter_start(kernel: str | None) -> None:
    """Arm the library's kernel meter for the launches named `kernel` (None disarms)."""
    _check(lib().dd_meter_start(kernel.encode() if kernel else None), "dd_meter_start")


def meter_read() -> dict:
    """Totals since meter_start: dispatches, summed event-timed ms, algorithmic flops and bytes."""
    m = _Meter()
    _check(lib().dd_meter_read(C.byref(m)), "dd_meter_read")
    return {"launches": m.launches, "total_ms": m.total_ms, "flops": m.flops, "bytes": m.bytes}


def autotune_report() -> str:
    """dd_autotune_report: the launch-mapping candidates per kernel family (chosen one starred)."""
    n = lib().dd_autotune_report(None, 0)
    buf = C.create_string_buffer(max(1, n) + 1)
    lib().dd_autotune_report(buf, len(buf))
    return buf.value.decode()


def library_path() -> str:
    return os.path.join(HERE, "libdd.so")


def lib():
    """Load libdd.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(path)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "dd_partition_ggg": ([P(_Csr), i32, C.c_uint64, vp, vp], i32),
        "dd_partition_ggg_noalloc": ([P(_Csr), i32, C.c_uint64, vp, vp], i32),
        "dd_setup": ([P(_Csr), vp, i32, i32, f64, i32, P(_Opts), vp, P(vp)], i32),
        "dd_update_values": ([vp, vp, vp], i32),
        "dd_setup_batch": ([P(_Csr), P(vp), P(i32), i32, i32, f64, i32, P(_Opts), vp, P(vp)], i32),
        "dd_apply": ([vp, vp, vp, i32, vp], i32),
        "dd_pcg": ([vp, vp, vp, i32, f64, i32, P(i32), P(f64), vp], i32),
        "dd_gmres": ([vp, vp, vp, i32, f64, i32, i32, P(i32), P(f64), vp], i32),
        "dd_spmv": ([vp, vp, vp, vp], i32),
        "dd_info": ([vp, P(_Info)], i32),
        "dd_phase_name": ([i32], C.c_char_p),
        "dd_destroy": ([vp], None),
        "dd_trim_device_cache": ([], i32),
        "dd_strerror": ([C.c_int], C.c_char_p),
        "dd_subdomain_count": ([vp, i32, P(i32)], i32),
        "dd_subdomain_sizes": ([vp, i32, vp], i32),
        "dd_subdomain_sets": ([vp, i32, i32, vp, vp, vp], i32),
        "dd_subdomain_eigs": ([vp, i32, i32, vp], i32),
        "dd_subdomain_basis": ([vp, i32, i32, vp], i32),
        "dd_subdomain_sigma1": ([vp, i32, vp], i32),
        "dd_extract_local": ([P(_Csr), vp, i32, i32, i32, vp, vp, vp, vp], i32),
        "dd_subdomain_eig_stats": ([vp, i32, vp, vp], i32),
        "dd_model_create": ([C.c_uint64, P(vp)], i32),
        "dd_model_add_samples": ([vp, vp, vp], i32),
        "dd_model_train": ([vp, i32, f64, vp, vp], i32),
        "dd_model_params": ([vp, vp, P(i32)], i32),
        "dd_model_set_params": ([vp, vp, i32], i32),
        "dd_model_forward": ([vp, vp, i64, vp, vp], i32),
        "dd_model_loss_grad": ([vp, vp, vp, vp, i64, vp, vp, vp], i32),
        "dd_model_samples": ([vp, P(i64), vp, vp, vp], i32),
        "dd_model_destroy": ([vp], None),
        "dd_coarse_matrix": ([vp, i32, vp, i64], i32),
        "dd_meter_start": ([C.c_char_p], i32),
        "dd_meter_read": ([P(_Meter)], i32),
        "dd_autotune_report": ([C.c_char_p, i64], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _LIB = L
    return L


def exported_symbols() -> list[str]:
    return ["dd_partition_ggg", "dd_partition_ggg_noalloc", "dd_setup", "dd_update_values", "dd_setup_batch", "dd_apply", "dd_pcg", "dd_gmres", "dd_spmv", "dd_info", "dd_phase_name",
            "dd_destroy", "dd_trim_device_cache", "dd_strerror", "dd_subdomain_count", "dd_subdomain_sizes", "dd_subdomain_sets",
            "dd_subdomain_eigs", "dd_subdomain_basis", "dd_subdomain_sigma1", "dd_coarse_matrix", "dd_extract_local",
            "dd_subdomain_eig_stats", "dd_model_create", "dd_model_add_samples", "dd_model_train", "dd_model_params",
            "dd_model_set_params", "dd_model_forward", "dd_model_loss_grad", "dd_model_samples", "dd_model_destroy",
            "dd_meter_start", "dd_meter_read", "dd_autotune_report"]


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


class DeviceCSR:
    """CSR matrix resident on the GPU (int32 indices, FP64 values, full symmetric storage)."""

    def __init__(self, n, rowptr, colind, val, device="cuda"):
        import torch
        self.n = int(n)
        self.rowptr = torch.as_tensor(np.asarray(rowptr, dtype=np.int32)).to(device)
        self.colind = torch.as_tensor(np.asarray(colind, dtype=np.int32)).to(device)
        self.val = torch.as_tensor(np.asarray(val, dtype=np.float64)).to(device)
        self.nnz = int(self.colind.numel())

    @classmethod
    def from_workload(cls, A, device="cuda"):
        return cls(A.n, A.rowptr, A.colind, A.val, device)

    def cstruct(self) -> _Csr:
        return _Csr(self.n, self.nnz, self.rowptr.data_ptr(), self.colind.data_ptr(), self.val.data_ptr())


def _check(code: int, what: str, allow_warn: bool = True) -> int:
    if code < 0 or (code > 0 and not allow_warn):
        raise DDError(code, what)
    return code


def trim_device_cache() -> None:
    """dd_trim_device_cache: return the library's cached device memory to the runtime."""
    _check(lib().dd_trim_device_cache(), "dd_trim_device_cache")


def partition_ggg(A: DeviceCSR, N: int, seed: int):
    import torch
    part = torch.empty(A.n, dtype=torch.int32, device=A.val.device)
    cs = A.cstruct()
    _check(lib().dd_partition_ggg(C.byref(cs), N, seed, _ptr(part), _stream()), "dd_partition_ggg")
    return part


MODEL_NFEAT = 8
MODEL_NPARAM = 8 * 32 + 32 + 32 * 32 + 32 + 32 + 1 + 2 * 8


class WarmStartModel:
    """dd_model: the network that weights the boundary nodes of the start block of
    the block eigensolver; trained on the GPU from the kept eigenvectors of setups."""

    def __init__(self, seed: int = 0):
        h = C.c_void_p()
        _check(lib().dd_model_create(int(seed), C.byref(h)), "dd_model_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dd_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_samples(self, pre) -> None:
        _check(lib().dd_model_add_samples(self._h, pre._h, _stream()), "dd_model_add_samples")

    def train(self, epochs: int, lr: float = 1e-2) -> np.ndarray:
        loss = np.zeros(max(1, epochs))
        _check(lib().dd_model_train(self._h, int(epochs), float(lr), loss.ctypes.data_as(C.c_void_p), _stream()),
               "dd_model_train")
        return loss[:epochs]

    def params(self) -> np.ndarray:
        out = np.zeros(MODEL_NPARAM)
        n = C.c_int32()
        _check(lib().dd_model_params(self._h, out.ctypes.data_as(C.c_void_p), C.byref(n)), "dd_model_params")
        return out[:n.value]

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(p, dtype=np.float64)
        _check(lib().dd_model_set_params(self._h, p.ctypes.data_as(C.c_void_p), p.size), "dd_model_set_params")

    def forward(self, feats):
        import torch
        f = torch.as_tensor(np.ascontiguousarray(feats, dtype=np.float64), device="cuda")
        out = torch.empty(f.shape[0], dtype=torch.float64, device="cuda")
        _check(lib().dd_model_forward(self._h, _ptr(f), f.shape[0], _ptr(out), _stream()), "dd_model_forward")
        return out.cpu().numpy()

    def loss_grad(self, feats, target, weight):
        import torch
        t = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda") for a in (feats, target, weight)]
        loss = np.zeros(1)
        grad = np.zeros(MODEL_NPARAM - 2 * MODEL_NFEAT)
        _check(lib().dd_model_loss_grad(self._h, _ptr(t[0]), _ptr(t[1]), _ptr(t[2]), t[1].numel(),
                                        loss.ctypes.data_as(C.c_void_p), grad.ctypes.data_as(C.c_void_p),
                                        _stream()), "dd_model_loss_grad")
        return float(loss[0]), grad

    def samples(self):
        n = C.c_int64()
        _check(lib().dd_model_samples(self._h, C.byref(n), None, None, None), "dd_model_samples")
        f, t, w = np.zeros((n.value, MODEL_NFEAT)), np.zeros(n.value), np.zeros(n.value)
        _check(lib().dd_model_samples(self._h, C.byref(n), f.ctypes.data_as(C.c_void_p), t.ctypes.data_as(C.c_void_p),
                                      w.ctypes.data_as(C.c_void_p)), "dd_model_samples")
        return f, t, w


def extract_local(A: DeviceCSR, part, N: int, overlap: int, i: int):
    """dd_extract_local: (sizes (n_I, n_Gamma, n_Delta), A_ii, X_i) of subdomain i as the setup forms them."""
    import torch
    part = torch.as_tensor(part, dtype=torch.int32).to(A.val.device).contiguous()
    cs = A.cstruct()
    sz = np.zeros(3, dtype=np.int32)
    _check(lib().dd_extract_local(C.byref(cs), _ptr(part), N, overlap, i, sz.ctypes.data_as(C.c_void_p), None,
                                  None, _stream()), "dd_extract_local")
    ni, nt = int(sz[0] + sz[1]), int(sz.sum())
    Aii = np.zeros(ni * ni)
    X = np.zeros(ni * nt)
    _check(lib().dd_extract_local(C.byref(cs), _ptr(part), N, overlap, i, None, Aii.ctypes.data_as(C.c_void_p),
                                  X.ctypes.data_as(C.c_void_p), _stream()), "dd_extract_local")
    return tuple(int(v) for v in sz), Aii.reshape(ni, ni).T.copy(), X.reshape(nt, ni).T.copy()


class Preconditioner:
    """Handle of dd_setup: the additive Schwarz preconditioner with `levels`
    levels (2 = fine + coarse E; more levels recurse on E, coarsening the
    subdomain graph by `coarsen`); schwarz=DD_SCHWARZ_DEFLATED for the
    deflated variant (solve with gmres)."""

    def __init__(self, A: DeviceCSR, part, N: int, overlap: int, tau: float, levels: int = 2,
                 local_prec: int = DD_FP64, select: int = DD_SEL_THRESHOLD, nev_cap: int = 0,
                 validate: bool = False, coarsen: int = 0, schwarz: int = DD_SCHWARZ_ADDITIVE,
                 eig_solver: int = DD_EIG_DENSE, lobpcg_maxit: int = 0, lobpcg_tol: float = 0.0,
                 warm_start: int = DD_START_RANDOM, seed: int = 0, model=None, graph_pcg: int = 0):
        import torch
        self.A = A
        self.n = A.n
        part = torch.as_tensor(part, dtype=torch.int32).to(A.val.device)
        opts = _opts(local_prec, select, nev_cap, validate, coarsen, schwarz, eig_solver, lobpcg_maxit, lobpcg_tol,
                     warm_start, seed, model, graph_pcg)
        self._model = model
        h = C.c_void_p()
        cs = A.cstruct()
        self.setup_status = _check(
            lib().dd_setup(C.byref(cs), _ptr(part), N, overlap, float(tau), levels, C.byref(opts), _stream(),
                           C.byref(h)), "dd_setup")
        self._h = h
        self.nsys = 1

    @classmethod
    def batch(cls, As, parts, Ns, overlap: int, tau: float, levels: int = 2, local_prec: int = DD_FP64,
              select: int = DD_SEL_THRESHOLD, nev_cap: int = 0, validate: bool = False, coarsen: int = 0,
              schwarz: int = DD_SCHWARZ_ADDITIVE, eig_solver: int = DD_EIG_DENSE, lobpcg_maxit: int = 0,
              lobpcg_tol: float = 0.0, warm_start: int = DD_START_RANDOM, seed: int = 0, model=None,
              graph_pcg: int = 0):
        """dd_setup_batch: independent systems As[j] (DeviceCSR) with partitions
        parts[j] into Ns[j] parts, one handle over their block-diagonal union.
        Vectors are the systems concatenated; pcg returns per-system counts."""
        import torch
        k = len(As)
        dev = As[0].val.device
        tparts = [torch.as_tensor(p, dtype=torch.int32).to(dev).contiguous() for p in parts]
        csrs = (_Csr * k)(*[A.cstruct() for A in As])
        pp = (C.c_void_p * k)(*[t.data_ptr() for t in tparts])
        ns = (C.c_int32 * k)(*[int(x) for x in Ns])
        opts = _opts(local_prec, select, nev_cap, validate, coarsen, schwarz, eig_solver, lobpcg_maxit, lobpcg_tol,
                     warm_start, seed, model, graph_pcg)
        h = C.c_void_p()
        self = cls.__new__(cls)
        self._model = model
        self.setup_status = _check(
            lib().dd_setup_batch(csrs, pp, ns, k, overlap, float(tau), levels, C.byref(opts), _stream(), C.byref(h)),
            "dd_setup_batch")
        self._h = h
        self.nsys = k
        self.sys_n = [A.n for A in As]
        self.n = sum(self.sys_n)
        self.A = None
        self._batch_nnz = sum(A.nnz for A in As)
        self._dev = dev
        self._keep = tparts
        return self

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_values(self, val):
        """dd_update_values: new matrix values (same pattern, CSR order), whole setup redone.
        A batch handle takes the values of all systems concatenated (system after system)."""
        import torch
        if self.A is None:
            val = torch.as_tensor(val, dtype=torch.float64).to(self._dev).contiguous()
            if val.numel() != self._batch_nnz:
                raise ValueError("update_values: expected the nnz values of all systems")
            self.setup_status = _check(lib().dd_update_values(self._h, _ptr(val), _stream()), "dd_update_values")
            self._keep_val = val
            return self.setup_status
        val = torch.as_tensor(val, dtype=torch.float64).to(self.A.val.device).contiguous()
        if val.numel() != self.A.val.numel():
            raise ValueError("update_values: expected nnz values")
        self.setup_status = _check(lib().dd_update_values(self._h, _ptr(val), _stream()), "dd_update_values")
        A = DeviceCSR.__new__(DeviceCSR)
        A.n, A.rowptr, A.colind, A.val, A.nnz = self.A.n, self.A.rowptr, self.A.colind, val, self.A.nnz
        self.A = A
        return self.setup_status

    # ---- solve phase ----
    # Vectors are 1-D (n) or 2-D (n, nrhs); the C-ABI takes column-major n x nrhs,
    # i.e. the storage of the transposed (nrhs, n) tensor.
    @staticmethod
    def _cm(t):
        return t.t().contiguous() if t.dim() == 2 else t.contiguous()

    @staticmethod
    def _uncm(t, two_d):
        return t.t() if two_d else t

    def apply(self, r):
        import torch
        rc = self._cm(r)
        z = torch.empty_like(rc)
        nrhs = 1 if r.dim() == 1 else r.shape[1]
        _check(lib().dd_apply(self._h, _ptr(rc), _ptr(z), nrhs, _stream()), "dd_apply")
        return self._uncm(z, r.dim() == 2)

    def pcg(self, b, x0=None, rtol: float = 1e-8, maxit: int = 1000):
        """dd_pcg; iters and relres hold nsys entries per right-hand side (system j of RHS k at k*nsys + j)."""
        import torch
        bc = self._cm(b)
        x = torch.zeros_like(bc) if x0 is None else self._cm(x0).clone()
        nrhs = 1 if b.dim() == 1 else b.shape[1]
        its = (C.c_int32 * (nrhs * self.nsys))()
        rr = (C.c_double * (nrhs * self.nsys))()
        code = _check(lib().dd_pcg(self._h, _ptr(bc), _ptr(x), nrhs, rtol, maxit, its, rr, _stream()), "dd_pcg")
        return self._uncm(x, b.dim() == 2), list(its), list(rr), code

    def gmres(self, b, x0=None, rtol: float = 1e-8, maxit: int = 1000, restart: int = 30):
        """dd_gmres: right-preconditioned GMRES(restart), flexible with more than two levels."""
        import torch
        bc = self._cm(b)
        x = torch.zeros_like(bc) if x0 is None else self._cm(x0).clone()
        nrhs = 1 if b.dim() == 1 else b.shape[1]
        its = (C.c_int32 * nrhs)()
        rr = (C.c_double * nrhs)()
        code = _check(lib().dd_gmres(self._h, _ptr(bc), _ptr(x), nrhs, rtol, maxit, restart, its, rr, _stream()),
                      "dd_gmres")
        return self._uncm(x, b.dim() == 2), list(its), list(rr), code

    def spmv(self, x):
        import torch
        y = torch.empty_like(x)
        _check(lib().dd_spmv(self._h, _ptr(x), _ptr(y), _stream()), "dd_spmv")
        return y

    # ---- diagnostics and inspection ----
    def info(self) -> dict:
        inf = _Info()
        _check(lib().dd_info(self._h, C.byref(inf)), "dd_info")
        L = lib()
        return {
            "levels": inf.levels, "N": list(inf.N), "n": list(inf.n), "n_C": inf.n_C,
            "grid_complexity": inf.grid_complexity, "p_min": inf.p_min, "p_max": inf.p_max,
            "p_hist": list(inf.p_hist), "k_c": inf.k_c,
            "fp32_fallbacks": inf.fp32_fallbacks, "eig_maxit_hits": inf.eig_maxit_hits,
            "eig_iters_max": inf.eig_iters_max, "eig_iters_mean": inf.eig_iters_mean,
            "eig_resid_max": inf.eig_resid_max,
            "phase_ms": {L.dd_phase_name(i).decode(): inf.phase_ms[i] for i in range(DD_NPHASE)},
            "last_iters": inf.last_iters, "last_relres": inf.last_relres, "device_bytes": inf.device_bytes,
            "coarse_factor_bytes": inf.coarse_factor_bytes,
        }

    def count(self, level=0) -> int:
        N = C.c_int32()
        _check(lib().dd_subdomain_count(self._h, level, C.byref(N)), "dd_subdomain_count")
        return N.value

    def sizes(self, level=0) -> np.ndarray:
        N = self.count(level)
        out = np.zeros(5 * N, dtype=np.int32)
        _check(lib().dd_subdomain_sizes(self._h, level, out.ctypes.data_as(C.c_void_p)), "dd_subdomain_sizes")
        return out.reshape(N, 5)

    def sets(self, i, level=0):
        nI, nG, nD = (int(v) for v in self.sizes(level)[i, :3])
        I, G, D = (np.zeros(k, dtype=np.int32) for k in (nI, nG, nD))
        _check(lib().dd_subdomain_sets(self._h, level, i, I.ctypes.data_as(C.c_void_p), G.ctypes.data_as(C.c_void_p),
                                       D.ctypes.data_as(C.c_void_p)), "dd_subdomain_sets")
        return I, G, D

    def eigs(self, i, level=0) -> np.ndarray:
        p = int(self.sizes(level)[i, 3])
        mu = np.zeros(p)
        _check(lib().dd_subdomain_eigs(self._h, level, i, mu.ctypes.data_as(C.c_void_p)), "dd_subdomain_eigs")
        return mu

    def basis(self, i, level=0) -> np.ndarray:
        nI, p = int(self.sizes(level)[i, 0]), int(self.sizes(level)[i, 3])
        Z = np.zeros(nI * p)
        _check(lib().dd_subdomain_basis(self._h, level, i, Z.ctypes.data_as(C.c_void_p)), "dd_subdomain_basis")
        return Z.reshape(p, nI).T.copy()

    def eig_stats(self, level=0):
        """dd_subdomain_eig_stats: block eigensolver iterations and final residual per subdomain."""
        N = self.count(level)
        it = np.zeros(N, dtype=np.int32)
        rr = np.zeros(N)
        _check(lib().dd_subdomain_eig_stats(self._h, level, it.ctypes.data_as(C.c_void_p),
                                            rr.ctypes.data_as(C.c_void_p)), "dd_subdomain_eig_stats")
        return it, rr

    def sigma1(self, level=0) -> np.ndarray:
        out = np.zeros(self.count(level))
        _check(lib().dd_subdomain_sigma1(self._h, level, out.ctypes.data_as(C.c_void_p)), "dd_subdomain_sigma1")
        return out

    def coarse_matrix(self, level=0, max_n=4096) -> np.ndarray:
        nC = self.info()["n_C"]
        E = np.zeros(nC * nC)
        _check(lib().dd_coarse_matrix(self._h, level, E.ctypes.data_as(C.c_void_p), max_n), "dd_coarse_matrix")
        return E.reshape(nC, nC).T.copy()
