"""cfmm: complex-coordinate fast multipole method on MI355X (gfx950).

Thin ctypes binding over the C-ABI in include/cfmm.h: argument marshalling
only, every step of the evaluation runs in the HIP library libcfmm.so.
PyTorch supplies device memory and streams.  Importing this package without
the built library raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcfmm.so")

CFMM_OK = 0
CFMM_EINVAL = -1
CFMM_ENOTSUP = -2
CFMM_EGEOMETRY = -3
CFMM_ENOMEM = -4
CFMM_EHIP = -5
CFMM_ERANGE = -6

LAPLACE = 0
HELMHOLTZ = 1
FP64 = 0
MIXED = 1

STAGES = ("gather", "p2m", "m2m", "m2l", "l2l", "l2p_m2p", "p2p", "eval")

_ERRNAMES = {CFMM_EINVAL: "EINVAL", CFMM_ENOTSUP: "ENOTSUP", CFMM_EGEOMETRY: "EGEOMETRY",
             CFMM_ENOMEM: "ENOMEM", CFMM_EHIP: "EHIP", CFMM_ERANGE: "ERANGE"}


class CfmmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cfmm error {_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


# smallest tolerances the library accepts (include/cfmm.h)
TOL_MIN = {(2, "laplace"): 1e-12, (2, "helmholtz"): 1e-12, (3, "laplace"): 1e-12, (3, "helmholtz"): 1e-10}
MIXED_TOL_MIN = 1e-6
STATIC_MAX = 1 << 22            # complex values of cfmm_eval_static's staging


class PlanDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("kernel", ctypes.c_int), ("wavenumber", ctypes.c_double),
                ("tol", ctypes.c_double), ("n_src", ctypes.c_int64), ("src", ctypes.c_void_p),
                ("n_trg", ctypes.c_int64), ("trg", ctypes.c_void_p),
                ("points_on_device", ctypes.c_int), ("precision", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("leaf_size", ctypes.c_int),
                ("separation", ctypes.c_int), ("m2l_form", ctypes.c_int)]


_lib = None


def lib():
    """The loaded libcfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2509_05458_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32p, i64p, u64p = (ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_uint64))
        L.cfmm_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(PlanDesc)]
        L.cfmm_eval.argtypes = [vp, vp, vp, ctypes.c_int]
        L.cfmm_eval_static.argtypes = [vp, vp, vp]
        L.cfmm_eval_layer.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int]
        L.cfmm_sync.argtypes = [vp]
        L.cfmm_destroy.argtypes = [vp]
        L.cfmm_plan_bytes.argtypes = [vp]
        L.cfmm_plan_bytes.restype = i64
        L.cfmm_last_error.restype = ctypes.c_char_p
        L.cfmm_plan_info.argtypes = [vp, i64p]
        L.cfmm_plan_m2l_work.argtypes = [vp, i64p]
        L.cfmm_plan_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.cfmm_plan_nterms.argtypes = [vp, ctypes.c_int]
        L.cfmm_plan_near_work.argtypes = [vp, i64p]
        L.cfmm_plan_export_tree.argtypes = [vp, i64p, u64p, i32p, i32p, i32p, i32p, i32p, i32p, u64p]
        L.cfmm_plan_export_list.argtypes = [vp, ctypes.c_int, i32p, i32p, i64p]
        L.cfmm_plan_export_centers.argtypes = [vp, vp]
        L.cfmm_plan_export_expansions.argtypes = [vp, vp, vp, i64p, i64p]
        L.cfmm_set_profiling.argtypes = [vp, ctypes.c_int]
        L.cfmm_ring_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        L.cfmm_stage_ms.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.cfmm_htree_build.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64, u64p, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int]
        L.cfmm_htree_sizes.argtypes = [vp, i64p]
        L.cfmm_htree_export.argtypes = [vp, i32p, i32p, i32p, i32p, i32p, i32p, u64p]
        L.cfmm_htree_export_list.argtypes = [vp, ctypes.c_int, i32p, i32p]
        L.cfmm_htree_free.argtypes = [vp]
        L.cfmm_nterms.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_double, ctypes.c_int]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != CFMM_OK:
        raise CfmmError(rc, lib().cfmm_last_error().decode())


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _as_points(x, name):
    """(keep-alive object, pointer, n, dim, on_device) of complex128 points [n, dim]."""
    if _is_torch(x) and x.is_cuda:
        import torch
        if x.dtype != torch.complex128 or x.dim() != 2:
            raise ValueError(f"{name}: expected a complex128 CUDA tensor [n, dim]")
        x = x.contiguous()
        return x, x.data_ptr(), x.shape[0], x.shape[1], True
    a = np.ascontiguousarray(x, dtype=np.complex128)
    if a.ndim != 2:
        raise ValueError(f"{name}: expected a complex array [n, dim]")
    return a, a.ctypes.data, a.shape[0], a.shape[1], False


class Plan:
    """A complex-coordinate FMM plan for u_i = sum_j G(x_i, y_j) sigma_j.

    points: complex128 sources [n_src, dim] (numpy on the host, or a torch
    CUDA tensor).  targets: optional complex128 [n_trg, dim] on the same side;
    without it the targets are the sources and the self term is left out.
    m2l_form: 3D Laplace M2L form, "auto" (point and shoot where it applies)
    or "direct" (the addition theorem for every pair).
    Evaluate with ``plan(sigma)`` for any number of densities.
    """

    def __init__(self, points, kernel: str = "helmholtz", kappa: float = 0.0,
                 tol: float = 1e-6, precision: str = "fp64", leaf_size: int = 0,
                 separation: int = 0, stream=None, targets=None, m2l_form: str = "auto"):
        L = lib()
        self._handle = ctypes.c_void_p()
        src, sptr, n, dim, on_dev = _as_points(points, "points")
        trg, tptr, nt = None, None, 0
        if targets is not None:
            trg, tptr, nt, tdim, t_dev = _as_points(targets, "targets")
            if tdim != dim or t_dev != on_dev:
                raise ValueError("targets must have the sources' dimension and live on the same side")
        if stream is None and on_dev:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        d = PlanDesc(dim=dim, kernel={"laplace": LAPLACE, "helmholtz": HELMHOLTZ}[kernel],
                     wavenumber=float(kappa), tol=float(tol), n_src=n, src=sptr,
                     n_trg=nt, trg=tptr, points_on_device=1 if on_dev else 0,
                     precision={"fp64": FP64, "mixed": MIXED}[precision],
                     stream=stream or 0, leaf_size=int(leaf_size), separation=int(separation),
                     m2l_form={"auto": 0, "direct": 1}[m2l_form])
        _check(L.cfmm_plan(ctypes.byref(self._handle), ctypes.byref(d)))
        del src, trg
        self.n = n
        self.n_out = nt if targets is not None else n
        self.dim, self.kernel, self.kappa, self.tol = dim, kernel, kappa, tol
        self.precision = precision
        self.stream = stream

    # ----------------------------------------------------------- evaluation
    def _check_tensor(self, x, n, name):
        import torch
        if not (_is_torch(x) and x.is_cuda and x.dtype == torch.complex128 and x.is_contiguous()
                and x.numel() == n):
            raise ValueError(f"{name}: expected a contiguous complex128 CUDA tensor of {n} elements")

    def eval_into(self, sigma, out) -> None:
        """Asynchronous device evaluation on the plan's stream: sigma [n_src]
        and out [n_out] are contiguous complex128 CUDA tensors.  The caller
        orders the plan's stream against the streams that produce sigma and
        consume out (the plan's stream is the current stream at plan time
        unless one was given)."""
        self._check_tensor(sigma, self.n, "sigma")
        self._check_tensor(out, self.n_out, "out")
        _check(lib().cfmm_eval(self._handle, sigma.data_ptr(), out.data_ptr(), 1))

    def __call__(self, sigma):
        L = lib()
        if _is_torch(sigma):
            import torch
            s = sigma.contiguous()
            self._check_tensor(s, self.n, "sigma")
            out = torch.empty(self.n_out, dtype=torch.complex128, device=s.device)
            cur = torch.cuda.current_stream(s.device)
            ps = torch.cuda.ExternalStream(self.stream or 0, device=s.device) \
                if (self.stream or 0) != cur.cuda_stream else cur
            if ps is not cur:
                ps.wait_stream(cur)           # sigma and out were made on the current stream
            _check(L.cfmm_eval(self._handle, s.data_ptr(), out.data_ptr(), 1))
            if ps is not cur:
                cur.wait_stream(ps)           # the caller reads out on the current stream
                s.record_stream(ps)
                out.record_stream(ps)
            return out
        s = np.ascontiguousarray(sigma, dtype=np.complex128).reshape(-1)
        if s.shape[0] != self.n:
            raise ValueError(f"sigma: expected {self.n} values, got {s.shape[0]}")
        out = np.empty(self.n_out, dtype=np.complex128)
        _check(L.cfmm_eval(self._handle, s.ctypes.data, out.ctypes.data, 0))
        return out

    def eval_layer(self, charge=None, dipole=None, potential: bool = True, gradient: bool = False):
        """Layer potentials (cfmm_eval_layer, dim 3 Laplace): charges sigma
        [n_src] and/or dipole vectors v [n_src, 3] (v = tau nu); returns
        (u [n_out] or None, grad u [n_out, 3] or None).  numpy arrays run on
        the host path, CUDA tensors on the device (asynchronous; call sync())."""
        dev = (charge is not None and _is_torch(charge)) or (dipole is not None and _is_torch(dipole))
        if dev:
            import torch
            d = (charge if charge is not None else dipole).device
            q = None if charge is None else charge.contiguous()
            v = None if dipole is None else dipole.contiguous()
            if q is not None:
                self._check_tensor(q, self.n, "charge")
            if v is not None:
                self._check_tensor(v, 3 * self.n, "dipole")
            u = torch.empty(self.n_out, dtype=torch.complex128, device=d) if potential else None
            g = torch.empty((self.n_out, 3), dtype=torch.complex128, device=d) if gradient else None
            _check(lib().cfmm_eval_layer(self._handle, None if q is None else q.data_ptr(),
                                         None if v is None else v.data_ptr(), None if u is None else u.data_ptr(),
                                         None if g is None else g.data_ptr(), 1))
            return u, g
        q = None if charge is None else np.ascontiguousarray(charge, dtype=np.complex128).reshape(self.n)
        v = None if dipole is None else np.ascontiguousarray(dipole, dtype=np.complex128).reshape(self.n, 3)
        u = np.empty(self.n_out, dtype=np.complex128) if potential else None
        g = np.empty((self.n_out, 3), dtype=np.complex128) if gradient else None
        _check(lib().cfmm_eval_layer(self._handle, None if q is None else q.ctypes.data,
                                     None if v is None else v.ctypes.data, None if u is None else u.ctypes.data,
                                     None if g is None else g.ctypes.data, 0))
        return u, g

    def eval_static(self, sigma):
        """Host evaluation staged through the library's static device buffer
        (cfmm_eval_static: no allocation; n_src + n_out <= STATIC_MAX)."""
        s = np.ascontiguousarray(sigma, dtype=np.complex128).reshape(-1)
        if s.shape[0] != self.n:
            raise ValueError(f"sigma: expected {self.n} values, got {s.shape[0]}")
        out = np.empty(self.n_out, dtype=np.complex128)
        _check(lib().cfmm_eval_static(self._handle, s.ctypes.data, out.ctypes.data))
        return out

    def sync(self):
        _check(lib().cfmm_sync(self._handle))

    # -------------------------------------------------------------- queries
    @property
    def nbytes(self) -> int:
        return int(lib().cfmm_plan_bytes(self._handle))

    def info(self) -> dict:
        a = np.zeros(20, dtype=np.int64)
        _check(lib().cfmm_plan_info(self._handle, _ptr(a, ctypes.c_int64)))
        keys = ("nbox", "nleaf", "nlevels", "top_level", "n_list1", "n_list2", "n_list3",
                "n_list4", "p2p_pairs", "m2l_pairs", "max_p", "dim", "kernel", "separation",
                "leaf_size", "precision", "n_src", "n_trg", "n_points", "m2l_source_coefs")
        return {k: int(v) for k, v in zip(keys, a)}

    def m2l_work(self) -> dict:
        """3D Laplace M2L pairs and algorithmic flops by form (cfmm_plan_m2l_work)."""
        a = np.zeros(4, dtype=np.int64)
        _check(lib().cfmm_plan_m2l_work(self._handle, _ptr(a, ctypes.c_int64)))
        return {"direct_pairs": int(a[0]), "direct_flops": int(a[1]),
                "pns_pairs": int(a[2]), "pns_flops": int(a[3])}

    def timing(self) -> dict:
        """Wall-clock ms of the plan's phases (cfmm_plan_timing)."""
        a = np.zeros(7, dtype=np.float64)
        _check(lib().cfmm_plan_timing(self._handle, _ptr(a, ctypes.c_double)))
        keys = ("keys_sort", "topology", "centres_p", "lists", "tables", "check", "total")
        return {k: float(v) for k, v in zip(keys, a)}

    def near_work(self) -> dict:
        """Ordered near-field interactions and the kernel evaluations producing them."""
        a = np.zeros(2, dtype=np.int64)
        _check(lib().cfmm_plan_near_work(self._handle, _ptr(a, ctypes.c_int64)))
        return {"interactions": int(a[0]), "evaluations": int(a[1])}

    def nterms(self) -> list:
        return [int(lib().cfmm_plan_nterms(self._handle, l)) for l in range(self.info()["nlevels"])]

    def export_tree(self) -> dict:
        info = self.info()
        nb, npt = info["nbox"], info["n_points"]
        out = {"perm": np.zeros(npt, np.int64), "keys": np.zeros(npt, np.uint64)}
        for k in ("level", "parent", "child0", "nchild", "pbeg", "pend"):
            out[k] = np.zeros(nb, np.int32)
        out["prefix"] = np.zeros(nb, np.uint64)
        i32 = ctypes.c_int32
        _check(lib().cfmm_plan_export_tree(
            self._handle, _ptr(out["perm"], ctypes.c_int64), _ptr(out["keys"], ctypes.c_uint64),
            _ptr(out["level"], i32), _ptr(out["parent"], i32), _ptr(out["child0"], i32),
            _ptr(out["nchild"], i32), _ptr(out["pbeg"], i32), _ptr(out["pend"], i32),
            _ptr(out["prefix"], ctypes.c_uint64)))
        return out

    def export_list(self, which: int):
        nb = self.info()["nbox"]
        cnt = ctypes.c_int64()
        _check(lib().cfmm_plan_export_list(self._handle, which, None, None, ctypes.byref(cnt)))
        off = np.zeros(nb + 1, np.int32)
        idx = np.zeros(max(1, cnt.value), np.int32)
        _check(lib().cfmm_plan_export_list(self._handle, which, _ptr(off, ctypes.c_int32),
                                           _ptr(idx, ctypes.c_int32), None))
        return off, idx[:cnt.value]

    def export_centers(self) -> np.ndarray:
        nb = self.info()["nbox"]
        c = np.zeros((nb, self.dim), np.complex128)
        _check(lib().cfmm_plan_export_centers(self._handle, c.ctypes.data))
        return c

    def export_expansions(self):
        """(mpole, local, offsets) of the last evaluation (complex128 arrays)."""
        nb = self.info()["nbox"]
        off = np.zeros(nb, np.int64)
        cnt = ctypes.c_int64()
        _check(lib().cfmm_plan_export_expansions(self._handle, None, None,
                                                 _ptr(off, ctypes.c_int64), ctypes.byref(cnt)))
        mp = np.zeros(max(1, cnt.value), np.complex128)
        lc = np.zeros(max(1, cnt.value), np.complex128)
        _check(lib().cfmm_plan_export_expansions(self._handle, mp.ctypes.data, lc.ctypes.data,
                                                 None, None))
        return mp[:cnt.value], lc[:cnt.value], off

    def set_profiling(self, mode=True):
        """0/False off, 1/True every stage (stage_ms), 2 near-field ring and
        3 M2L-translation ring (ring_ms)."""
        _check(lib().cfmm_set_profiling(self._handle, int(mode)))

    def ring_ms(self):
        """(summed ms, evaluations) of the stage bracketed in profiling mode 2 or 3."""
        tot, cnt = ctypes.c_double(), ctypes.c_int()
        _check(lib().cfmm_ring_ms(self._handle, ctypes.byref(tot), ctypes.byref(cnt)))
        return tot.value, cnt.value

    def stage_ms(self) -> dict:
        out = {}
        v = ctypes.c_double()
        for i, name in enumerate(STAGES):
            _check(lib().cfmm_stage_ms(self._handle, i, ctypes.byref(v)))
            out[name] = v.value
        return out

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            lib().cfmm_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ host logic
def host_tree(dim: int, sorted_keys: np.ndarray, leaf_size: int, separation: int = 1,
              top: int = 0) -> dict:
    """The library's tree and Lists 1-4 from sorted Morton keys (no GPU needed)."""
    L = lib()
    keys = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    h = ctypes.c_void_p()
    _check(L.cfmm_htree_build(ctypes.byref(h), dim, keys.shape[0], _ptr(keys, ctypes.c_uint64),
                              leaf_size, separation, top))
    try:
        s = np.zeros(6, np.int64)
        _check(L.cfmm_htree_sizes(h, _ptr(s, ctypes.c_int64)))
        nb = int(s[0])
        out = {k: np.zeros(nb, np.int32) for k in ("level", "parent", "child0", "nchild", "pbeg", "pend")}
        out["prefix"] = np.zeros(nb, np.uint64)
        i32 = ctypes.c_int32
        _check(L.cfmm_htree_export(h, _ptr(out["level"], i32), _ptr(out["parent"], i32),
                                   _ptr(out["child0"], i32), _ptr(out["nchild"], i32),
                                   _ptr(out["pbeg"], i32), _ptr(out["pend"], i32),
                                   _ptr(out["prefix"], ctypes.c_uint64)))
        for q in range(4):
            off = np.zeros(nb + 1, np.int32)
            idx = np.zeros(max(1, int(s[1 + q])), np.int32)
            _check(L.cfmm_htree_export_list(h, q + 1, _ptr(off, i32), _ptr(idx, i32)))
            out[f"L{q + 1}"] = (off, idx[:int(s[1 + q])])
        return out
    finally:
        L.cfmm_htree_free(h)


def nterms(dim: int, kernel: str, kappa: float, w: float, separation: int, eps: float,
           pmax: int = 63) -> int:
    """Expansion length the plan uses for boxes of width w."""
    rc = lib().cfmm_nterms(dim, {"laplace": LAPLACE, "helmholtz": HELMHOLTZ}[kernel],
                           float(kappa), float(w), int(separation), float(eps), int(pmax))
    if rc < 0:
        _check(rc)
    return int(rc)
