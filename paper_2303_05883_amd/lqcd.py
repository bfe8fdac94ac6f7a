"""ctypes binding of liblqcd.so, the gfx950 Wilson/clover library (include/lqcd.h).

Argument marshalling only: every step of the operator and the solvers runs in
the library's HIP kernels. Arrays may be NumPy (host) or torch tensors on the
GPU (device); complex128 with the canonical layouts:

* spinor ``[Lt, Lz, Ly, Lx, 4, 3]``
* gauge  ``[Lt, Lz, Ly, Lx, 4, 3, 3]``

The library must have been built (``python -m paper_2303_05883_amd.build``);
importing this module without it raises at once.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblqcd.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE, ENOCONV, EBREAKDOWN, ENOTSU3, ESINGULAR = 0, -1, -2, -3, -4, -5, -6, -7, -8
F64, F32, F16 = 0, 1, 2
(D, DEE, DOO, DEO, DOE, DPREC_PAPER, DPREC_SCHUR, DEE_INV, DOO_INV, HOP_EO, HOP_OE) = range(11)
OPS = {"D": D, "DEE": DEE, "DOO": DOO, "DEO": DEO, "DOE": DOE, "DPREC_PAPER": DPREC_PAPER,
       "DPREC_SCHUR": DPREC_SCHUR, "DEE_INV": DEE_INV, "DOO_INV": DOO_INV, "HOP_EO": HOP_EO, "HOP_OE": HOP_OE}

EXPORTED = ["lqcd_create", "lqcd_destroy", "lqcd_set_gauge", "lqcd_set_clover", "lqcd_apply",
            "lqcd_default_params", "lqcd_solve", "lqcd_solve_batch", "lqcd_field_bytes", "lqcd_import",
            "lqcd_export", "lqcd_apply_native", "lqcd_autotune", "lqcd_set_hop_shape", "lqcd_get_hop_shape",
            "lqcd_apply_sap", "lqcd_solve_sap", "lqcd_stag_apply", "lqcd_stag_solve", "lqcd_stag_field_bytes",
            "lqcd_stag_import", "lqcd_stag_export", "lqcd_stag_hop_native", "lqcd_dwf_apply",
            "lqcd_dwf_solve", "lqcd_dwf_field_bytes", "lqcd_dwf_import", "lqcd_dwf_export", "lqcd_dwf_apply_native",
            "lqcd_mg_setup", "lqcd_mg_coarse_size", "lqcd_mg_restrict", "lqcd_mg_prolong", "lqcd_mg_coarse_apply",
            "lqcd_mg_apply", "lqcd_solve_mg", "lqcd_dwf_apply_schur", "lqcd_dwf_solve_eo", "lqcd_batch_autotune", "lqcd_batch_apply_schur", "lqcd_apply_native_noalloc", "lqcd_bandwidth_probe", "lqcd_strerror",
            "lqcd_last_error"]
STAG_OPS = {"D": 0, "SCHUR": 1}


class SolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("max_outer", C.c_int), ("inner_prec", C.c_int),
                ("inner_tol", C.c_double), ("check_every", C.c_int), ("use_graph", C.c_int),
                ("x0", C.c_void_p), ("on_device", C.c_int), ("reliable_update", C.c_int), ("even_odd", C.c_int)]


class SapParams(C.Structure):
    _fields_ = [("block", C.c_int * 4), ("ncycles", C.c_int), ("nmr", C.c_int)]


def sap_params(block=(4, 4, 4, 4), ncycles: int = 2, nmr: int = 4) -> SapParams:
    sp = SapParams()
    for k in range(4):
        sp.block[k] = int(block[k])
    sp.ncycles, sp.nmr = int(ncycles), int(nmr)
    return sp


class MgParams(C.Structure):
    _fields_ = [("agg", C.c_int * 4), ("nvec", C.c_int), ("setup_iters", C.c_int), ("sap", SapParams),
                ("coarse_tol", C.c_double), ("coarse_max_iter", C.c_int)]


def mg_params(agg=(4, 4, 4, 4), nvec: int = 8, setup_iters: int = 3, sap_block=(4, 4, 4, 4), ncycles: int = 2,
              nmr: int = 4, coarse_tol: float = 0.05, coarse_max_iter: int = 200) -> MgParams:
    mp = MgParams()
    for k in range(4):
        mp.agg[k] = int(agg[k])
    mp.nvec, mp.setup_iters = int(nvec), int(setup_iters)
    mp.sap = sap_params(sap_block, ncycles, nmr)
    mp.coarse_tol, mp.coarse_max_iter = float(coarse_tol), int(coarse_max_iter)
    return mp


class DwfParams(C.Structure):
    _fields_ = [("Ls", C.c_int), ("M5", C.c_double), ("mf", C.c_double), ("b5", C.c_double), ("c5", C.c_double)]


def dwf_params(Ls: int, M5: float, mf: float, b5: float = 1.0, c5: float = 0.0) -> DwfParams:
    d = DwfParams()
    d.Ls, d.M5, d.mf, d.b5, d.c5 = int(Ls), float(M5), float(mf), float(b5), float(c5)
    return d


class SolveStats(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("inner_iters", C.c_int), ("restarts", C.c_int),
                ("true_rel_resid", C.c_double), ("seconds_solve", C.c_double), ("seconds_setup", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LqcdError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the library (once). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2303_05883_amd.build`")
    # torch ships its own HIP runtime under the same soname; loading torch first
    # makes the library bind to that one, so that the process holds a single HIP
    # runtime and torch's streams and allocations are valid in library calls.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp, ip, dp = C.c_void_p, C.c_int, C.c_double
    lib.lqcd_create.argtypes = [C.POINTER(C.c_int), ip, vp, C.POINTER(vp)]
    lib.lqcd_destroy.argtypes = [vp]
    lib.lqcd_set_gauge.argtypes = [vp, vp, ip]
    lib.lqcd_set_clover.argtypes = [vp, dp, dp]
    lib.lqcd_apply.argtypes = [vp, ip, ip, vp, vp, ip]
    lib.lqcd_default_params.argtypes = [C.POINTER(SolveParams)]
    lib.lqcd_default_params.restype = None
    lib.lqcd_solve.argtypes = [vp, vp, vp, C.POINTER(SolveParams), C.POINTER(SolveStats)]
    lib.lqcd_solve_batch.argtypes = [C.POINTER(vp), C.POINTER(C.c_int), C.POINTER(vp), C.POINTER(vp), ip,
                                     C.POINTER(SolveParams), C.POINTER(SolveStats)]
    lib.lqcd_batch_autotune.argtypes = [C.POINTER(vp), C.POINTER(C.c_int), ip, ip, C.POINTER(C.c_int),
                                        C.POINTER(C.c_double)]
    lib.lqcd_batch_apply_schur.argtypes = [C.POINTER(vp), C.POINTER(C.c_int), ip, ip, C.POINTER(vp), C.POINTER(vp)]
    lib.lqcd_field_bytes.argtypes = [vp, ip]
    lib.lqcd_field_bytes.restype = C.c_size_t
    lib.lqcd_import.argtypes = [vp, ip, ip, vp, vp]
    lib.lqcd_export.argtypes = [vp, ip, ip, vp, vp]
    lib.lqcd_apply_native.argtypes = [vp, ip, ip, vp, vp]
    lib.lqcd_apply_native_noalloc.argtypes = [vp, ip, ip, vp, vp]
    lib.lqcd_autotune.argtypes = [vp, ip, C.c_char_p]
    lib.lqcd_set_hop_shape.argtypes = [vp, ip, ip, ip, ip, ip]
    lib.lqcd_get_hop_shape.argtypes = [vp, ip] + [C.POINTER(C.c_int)] * 4
    lib.lqcd_apply_sap.argtypes = [vp, C.POINTER(SapParams), vp, vp, ip]
    lib.lqcd_stag_apply.argtypes = [vp, ip, ip, dp, vp, vp, ip]
    lib.lqcd_stag_solve.argtypes = [vp, dp, vp, vp, C.POINTER(SolveParams), C.POINTER(SolveStats)]
    lib.lqcd_stag_field_bytes.argtypes = [vp, ip]
    lib.lqcd_stag_field_bytes.restype = C.c_size_t
    lib.lqcd_stag_import.argtypes = [vp, ip, ip, vp, vp]
    lib.lqcd_stag_export.argtypes = [vp, ip, ip, vp, vp]
    lib.lqcd_dwf_apply.argtypes = [vp, C.POINTER(DwfParams), ip, ip, vp, vp, ip]
    lib.lqcd_dwf_solve.argtypes = [vp, C.POINTER(DwfParams), vp, vp, C.POINTER(SolveParams), C.POINTER(SolveStats)]
    lib.lqcd_dwf_apply_schur.argtypes = [vp, C.POINTER(DwfParams), ip, ip, vp, vp, ip]
    lib.lqcd_dwf_solve_eo.argtypes = [vp, C.POINTER(DwfParams), vp, vp, C.POINTER(SolveParams), C.POINTER(SolveStats)]
    lib.lqcd_dwf_field_bytes.argtypes = [vp, ip, ip]
    lib.lqcd_dwf_field_bytes.restype = C.c_size_t
    lib.lqcd_dwf_import.argtypes = [vp, ip, ip, vp, vp]
    lib.lqcd_dwf_export.argtypes = [vp, ip, ip, vp, vp]
    lib.lqcd_dwf_apply_native.argtypes = [vp, C.POINTER(DwfParams), ip, ip, vp, vp, vp]
    lib.lqcd_stag_hop_native.argtypes = [vp, ip, ip, vp, vp]
    lib.lqcd_solve_sap.argtypes = [vp, vp, vp, C.POINTER(SolveParams), C.POINTER(SapParams), C.POINTER(SolveStats)]
    lib.lqcd_mg_setup.argtypes = [vp, C.POINTER(MgParams), vp, ip]
    lib.lqcd_mg_coarse_size.argtypes = [vp]
    lib.lqcd_mg_coarse_size.restype = C.c_size_t
    for name in ("lqcd_mg_restrict", "lqcd_mg_prolong", "lqcd_mg_coarse_apply", "lqcd_mg_apply"):
        getattr(lib, name).argtypes = [vp, vp, vp, ip]
    lib.lqcd_solve_mg.argtypes = [vp, vp, vp, C.POINTER(SolveParams), C.POINTER(SolveStats)]
    lib.lqcd_bandwidth_probe.argtypes = [vp, ip, C.c_size_t, ip, C.POINTER(C.c_double)]
    lib.lqcd_bandwidth_probe.restype = ip
    lib.lqcd_strerror.argtypes = [ip]
    lib.lqcd_strerror.restype = C.c_char_p
    lib.lqcd_last_error.argtypes = []
    lib.lqcd_last_error.restype = C.c_char_p
    for name in ("lqcd_create", "lqcd_destroy", "lqcd_set_gauge", "lqcd_set_clover", "lqcd_apply", "lqcd_solve",
                 "lqcd_solve_batch", "lqcd_import", "lqcd_export", "lqcd_apply_native", "lqcd_autotune",
                 "lqcd_set_hop_shape", "lqcd_get_hop_shape", "lqcd_apply_sap", "lqcd_solve_sap",
                 "lqcd_stag_apply", "lqcd_stag_solve", "lqcd_stag_import", "lqcd_stag_export",
                 "lqcd_stag_hop_native", "lqcd_dwf_apply", "lqcd_dwf_solve", "lqcd_dwf_import",
                 "lqcd_dwf_export", "lqcd_dwf_apply_native", "lqcd_mg_setup", "lqcd_mg_restrict", "lqcd_mg_prolong",
                 "lqcd_mg_coarse_apply", "lqcd_mg_apply", "lqcd_solve_mg", "lqcd_dwf_apply_schur",
                 "lqcd_dwf_solve_eo"):
        getattr(lib, name).restype = ip
    _lib = lib
    return lib


def _check(status: int, where: str, allow=()):
    if status != OK and status not in allow:
        lib = load()
        raise LqcdError(status, where, f"{lib.lqcd_strerror(status).decode()}: {lib.lqcd_last_error().decode()}")
    return status


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _ptr(a):
    """(pointer, on_device) of a contiguous complex128 array or tensor."""
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), 1 if a.is_cuda else 0
    if not (isinstance(a, np.ndarray) and a.flags.c_contiguous):
        raise ValueError("array must be a C-contiguous numpy array or torch tensor")
    return a.ctypes.data, 0


def default_params() -> SolveParams:
    p = SolveParams()
    load().lqcd_default_params(C.byref(p))
    return p


@dataclass
class Stats:
    outer_iters: int
    inner_iters: int
    restarts: int
    true_rel_resid: float
    seconds_solve: float
    seconds_setup: float
    status: int


def _torch_cuda():
    try:
        import torch
    except ImportError:
        return None
    return torch if torch.cuda.is_available() else None


class Lattice:
    """One lattice context: dims = (Lx, Ly, Lz, Lt), t_bc = -1 or +1.

    With torch on a GPU the context runs on a torch stream of its own
    (``self.stream``); every call orders it after torch's current stream on
    entry and orders torch's current stream after it on exit, so tensors can
    be passed freely. ``stream`` may instead give a hipStream_t handle.
    """

    def __init__(self, dims, t_bc: int = -1, stream=None):
        """stream: None (a torch stream of its own when torch sees a GPU), a
        torch.cuda.Stream (share it, e.g. across the lattices of one batched
        solve), or a raw hipStream_t handle."""
        lib = load()
        self.dims = tuple(int(d) for d in dims)
        arr = (C.c_int * 4)(*self.dims)
        h = C.c_void_p()
        self.stream = None
        if stream is not None and hasattr(stream, "cuda_stream"):
            # a torch stream, possibly shared with other lattices (batched solves)
            self.stream = stream
            stream = stream.cuda_stream
        elif stream is None:
            torch = _torch_cuda()
            if torch is not None:
                self.stream = torch.cuda.Stream()
                stream = self.stream.cuda_stream
        s = C.c_void_p(int(stream)) if stream is not None else None
        _check(lib.lqcd_create(arr, int(t_bc), s, C.byref(h)), "lqcd_create")
        self.handle = h
        self.lib = lib

    def _enter(self):
        if self.stream is not None:
            import torch
            self.stream.wait_stream(torch.cuda.current_stream())

    def _exit(self):
        if self.stream is not None:
            import torch
            torch.cuda.current_stream().wait_stream(self.stream)

    def _call(self, fn, *args):
        self._enter()
        try:
            return fn(*args)
        finally:
            self._exit()

    def close(self):
        if getattr(self, "handle", None):
            self.lib.lqcd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # set-up ----------------------------------------------------------------
    def set_gauge(self, U):
        p, dev = _ptr(U)
        _check(self._call(self.lib.lqcd_set_gauge, self.handle, p, dev), "lqcd_set_gauge")

    def set_clover(self, kappa: float, csw: float = 0.0):
        _check(self._call(self.lib.lqcd_set_clover, self.handle, float(kappa), float(csw)), "lqcd_set_clover")

    # operators -------------------------------------------------------------
    def apply(self, op, prec, x, out):
        op = OPS[op] if isinstance(op, str) else int(op)
        pi, di = _ptr(x)
        po, do = _ptr(out)
        if di != do:
            raise ValueError("in and out must both be host or both be device")
        _check(self._call(self.lib.lqcd_apply, self.handle, op, int(prec), pi, po, di), "lqcd_apply")
        return out

    def field_bytes(self, prec: int) -> int:
        return int(self.lib.lqcd_field_bytes(self.handle, int(prec)))

    def import_field(self, prec, parity, canon, native):
        _check(self._call(self.lib.lqcd_import, self.handle, int(prec), int(parity), _ptr(canon)[0],
                          _ptr(native)[0]), "lqcd_import")

    def export_field(self, prec, parity, native, canon):
        _check(self._call(self.lib.lqcd_export, self.handle, int(prec), int(parity), _ptr(native)[0],
                          _ptr(canon)[0]), "lqcd_export")

    def apply_native(self, op, prec, native_in, native_out):
        op = OPS[op] if isinstance(op, str) else int(op)
        _check(self._call(self.lib.lqcd_apply_native, self.handle, op, int(prec), _ptr(native_in)[0],
                          _ptr(native_out)[0]), "lqcd_apply_native")

    def apply_native_noalloc(self, op, prec, native_in, native_out):
        """apply_native without any device allocation (the library's static scratch)."""
        op = OPS[op] if isinstance(op, str) else int(op)
        _check(self._call(self.lib.lqcd_apply_native_noalloc, self.handle, op, int(prec), _ptr(native_in)[0],
                          _ptr(native_out)[0]), "lqcd_apply_native_noalloc")

    def apply_native_repeat(self, op, prec, ins, outs, reps: int):
        """reps launches of one native operator, cycling over the (in, out)
        pairs, enqueued back to back (one stream ordering for the whole loop)."""
        op = OPS[op] if isinstance(op, str) else int(op)
        pi = [_ptr(t)[0] for t in ins]
        po = [_ptr(t)[0] for t in outs]
        self._enter()
        try:
            for r in range(int(reps)):
                k = r % len(pi)
                _check(self.lib.lqcd_apply_native(self.handle, op, int(prec), pi[k], po[k]), "lqcd_apply_native")
        finally:
            self._exit()

    def set_hop_shape(self, prec: int, block: int = 256, split: int = 1, xcd_map: int = 1, nt: int = 0):
        _check(self.lib.lqcd_set_hop_shape(self.handle, int(prec), int(block), int(split), int(xcd_map), int(nt)),
               "lqcd_set_hop_shape")

    def get_hop_shape(self, prec: int):
        """(block, split, xcd_map, nt) of the hop launch shape in use for prec."""
        v = [C.c_int() for _ in range(4)]
        _check(self.lib.lqcd_get_hop_shape(self.handle, int(prec), *[C.byref(x) for x in v]), "lqcd_get_hop_shape")
        return tuple(x.value for x in v)

    def bandwidth_probe(self, kind: int, nbytes: int = 1 << 30, reps: int = 5) -> float:
        """Best-of-reps GB/s of a read-only stream (kind 0) or a copy (kind 1)
        of nbytes on this context's GPU."""
        g = C.c_double(0.0)
        _check(self._call(self.lib.lqcd_bandwidth_probe, self.handle, int(kind), int(nbytes), int(reps), C.byref(g)),
               "lqcd_bandwidth_probe")
        return g.value

    def autotune(self, prec: int, path: str | None = None):
        _check(self._call(self.lib.lqcd_autotune, self.handle, int(prec), path.encode() if path else None),
               "lqcd_autotune")

    # solver ----------------------------------------------------------------
    def solve(self, b, x, tol=1e-10, inner_prec=F64, inner_tol=0.0, max_iter=100000, max_outer=100,
              check_every=8, use_graph=True, x0=None, raise_on_fail=True, reliable_update=False,
              even_odd=True) -> Stats:
        """D x = b; even_odd=False: FP64 BiCGStab on the full operator (no preconditioning)."""
        prm = default_params()
        pb, db = _ptr(b)
        px, dx = _ptr(x)
        if db != dx:
            raise ValueError("b and x must both be host or both be device")
        prm.tol, prm.inner_prec, prm.inner_tol = float(tol), int(inner_prec), float(inner_tol)
        prm.max_iter, prm.max_outer, prm.check_every = int(max_iter), int(max_outer), int(check_every)
        prm.use_graph, prm.on_device = int(bool(use_graph)), db
        prm.reliable_update = int(bool(reliable_update))
        prm.even_odd = int(bool(even_odd))
        if x0 is not None:
            prm.x0 = _ptr(x0)[0]
        st = SolveStats()
        status = self._call(self.lib.lqcd_solve, self.handle, pb, px, C.byref(prm), C.byref(st))
        if raise_on_fail:
            _check(status, "lqcd_solve")
        return Stats(st.outer_iters, st.inner_iters, st.restarts, st.true_rel_resid, st.seconds_solve,
                     st.seconds_setup, status)

    def apply_sap(self, eta, psi, block=(4, 4, 4, 4), ncycles=2, nmr=4):
        """psi = M eta, the FP32 SAP preconditioner (canonical full-lattice vectors)."""
        pi, di = _ptr(eta)
        po, do = _ptr(psi)
        if di != do:
            raise ValueError("eta and psi must both be host or both be device")
        sp = sap_params(block, ncycles, nmr)
        _check(self._call(self.lib.lqcd_apply_sap, self.handle, C.byref(sp), pi, po, di), "lqcd_apply_sap")
        return psi

    def solve_sap(self, b, x, block=(4, 4, 4, 4), ncycles=2, nmr=4, tol=1e-10, max_iter=10000, max_outer=20,
                  x0=None, raise_on_fail=True) -> Stats:
        """D x = b by FP64 flexible BiCGStab with the SAP preconditioner on the right."""
        prm = default_params()
        pb, db = _ptr(b)
        px, dx = _ptr(x)
        if db != dx:
            raise ValueError("b and x must both be host or both be device")
        prm.tol, prm.max_iter, prm.max_outer, prm.on_device = float(tol), int(max_iter), int(max_outer), db
        if x0 is not None:
            prm.x0 = _ptr(x0)[0]
        sp = sap_params(block, ncycles, nmr)
        st = SolveStats()
        status = self._call(self.lib.lqcd_solve_sap, self.handle, pb, px, C.byref(prm), C.byref(sp), C.byref(st))
        if raise_on_fail:
            _check(status, "lqcd_solve_sap")
        return Stats(st.outer_iters, st.inner_iters, st.restarts, st.true_rel_resid, st.seconds_solve,
                     st.seconds_setup, status)

    def mg_setup(self, start, **kw):
        """Multigrid setup from start vectors [nvec, Lt, Lz, Ly, Lx, 4, 3]; kw as mg_params."""
        ps, ds = _ptr(start)
        mp = mg_params(**kw)
        _check(self._call(self.lib.lqcd_mg_setup, self.handle, C.byref(mp), ps, ds), "lqcd_mg_setup")

    def mg_coarse_size(self) -> int:
        return int(self.lib.lqcd_mg_coarse_size(self.handle))

    def _mg_pair(self, name, a, b):
        pa, da = _ptr(a)
        pb, dbv = _ptr(b)
        if da != dbv:
            raise ValueError("both arguments must be host or both be device")
        _check(self._call(getattr(self.lib, name), self.handle, pa, pb, da), name)
        return b

    def mg_restrict(self, fine, coarse):
        return self._mg_pair("lqcd_mg_restrict", fine, coarse)

    def mg_prolong(self, coarse, fine):
        return self._mg_pair("lqcd_mg_prolong", coarse, fine)

    def mg_coarse_apply(self, x, y):
        return self._mg_pair("lqcd_mg_coarse_apply", x, y)

    def mg_apply(self, r, x):
        return self._mg_pair("lqcd_mg_apply", r, x)

    def solve_mg(self, b, x, tol=1e-10, max_iter=10000, max_outer=20, x0=None, raise_on_fail=True) -> Stats:
        """D x = b by FP64 flexible BiCGStab with the two-level multigrid preconditioner."""
        prm = default_params()
        pb, db = _ptr(b)
        px, dx = _ptr(x)
        if db != dx:
            raise ValueError("b and x must both be host or both be device")
        prm.tol, prm.max_iter, prm.max_outer, prm.on_device = float(tol), int(max_iter), int(max_outer), db
        if x0 is not None:
            prm.x0 = _ptr(x0)[0]
        st = SolveStats()
        status = self._call(self.lib.lqcd_solve_mg, self.handle, pb, px, C.byref(prm), C.byref(st))
        if raise_on_fail:
            _check(status, "lqcd_solve_mg")
        return Stats(st.outer_iters, st.inner_iters, st.restarts, st.true_rel_resid, st.seconds_solve,
                     st.seconds_setup, status)

    def stag_apply(self, op, prec, mass, x, out):
        """Staggered operator (STAG_OPS) on canonical colour-vector fields [Lt, Lz, Ly, Lx, 3]."""
        op = STAG_OPS[op] if isinstance(op, str) else int(op)
        pi, di = _ptr(x)
        po, do = _ptr(out)
        if di != do:
            raise ValueError("in and out must both be host or both be device")
        _check(self._call(self.lib.lqcd_stag_apply, self.handle, op, int(prec), float(mass), pi, po, di),
               "lqcd_stag_apply")
        return out

    def dwf_apply(self, Ls, M5, mf, prec, x, out, dag=False, b5=1.0, c5=0.0):
        """Moebius domain-wall D (or D^dag) on canonical 5-d fields [Ls, Lt, Lz, Ly, Lx, 4, 3]."""
        pi, di = _ptr(x)
        po, do = _ptr(out)
        if di != do:
            raise ValueError("in and out must both be host or both be device")
        d = dwf_params(Ls, M5, mf, b5, c5)
        _check(self._call(self.lib.lqcd_dwf_apply, self.handle, C.byref(d), int(bool(dag)), int(prec), pi, po, di),
               "lqcd_dwf_apply")
        return out

    def dwf_solve(self, Ls, M5, mf, b, x, tol=1e-10, max_iter=100000, max_outer=20, raise_on_fail=True, b5=1.0,
                  c5=0.0) -> Stats:
        """Moebius domain-wall D x = b by FP64 CG on the normal equations."""
        prm = default_params()
        pb, db = _ptr(b)
        px, dx = _ptr(x)
        if db != dx:
            raise ValueError("b and x must both be host or both be device")
        prm.tol, prm.max_iter, prm.max_outer, prm.on_device = float(tol), int(max_iter), int(max_outer), db
        d = dwf_params(Ls, M5, mf, b5, c5)
        st = SolveStats()
        status = self._call(self.lib.lqcd_dwf_solve, self.handle, C.byref(d), pb, px, C.byref(prm), C.byref(st))
        if raise_on_fail:
            _check(status, "lqcd_dwf_solve")
        return Stats(st.outer_iters, st.inner_iters, st.restarts, st.true_rel_resid, st.seconds_solve,
                     st.seconds_setup, status)

    def dwf_apply_schur(self, Ls, M5, mf, prec, x, out, dag=False, b5=1.0, c5=0.0):
        """The even-odd Schur complement S_ee (or its adjoint) on the even sites of canonical 5-d fields."""
        pi, di = _ptr(x)
        po, do = _ptr(out)
        if di != do:
            raise ValueError("in and out must both be host or both be device")
        d = dwf_params(Ls, M5, mf, b5, c5)
        _check(self._call(self.lib.lqcd_dwf_apply_schur, self.handle, C.byref(d), int(bool(dag)), int(prec), pi, po,
                          di), "lqcd_dwf_apply_schur")
        return out

    def dwf_solve_eo(self, Ls, M5, mf, b, x, tol=1e-10, max_iter=100000, max_outer=20, raise_on_fail=True, b5=1.0,
                     c5=0.0, inner_prec=F64, inner_tol=0.0) -> Stats:
        """Moebius domain-wall D x = b through the even-odd Schur complement and CG
        (FP64, or FP32 inner solves under FP64 defect correction with inner_prec=F32)."""
        prm = default_params()
        pb, db = _ptr(b)
        px, dx = _ptr(x)
        if db != dx:
            raise ValueError("b and x must both be host or both be device")
        prm.tol, prm.max_iter, prm.max_outer, prm.on_device = float(tol), int(max_iter), int(max_outer), db
        prm.inner_prec, prm.inner_tol = int(inner_prec), float(inner_tol)
        d = dwf_params(Ls, M5, mf, b5, c5)
        st = SolveStats()
        status = self._call(self.lib.lqcd_dwf_solve_eo, self.handle, C.byref(d), pb, px, C.byref(prm), C.byref(st))
        if raise_on_fail:
            _check(status, "lqcd_dwf_solve_eo")
        return Stats(st.outer_iters, st.inner_iters, st.restarts, st.true_rel_resid, st.seconds_solve,
                     st.seconds_setup, status)

    def dwf_field_bytes(self, prec: int, Ls: int) -> int:
        return int(self.lib.lqcd_dwf_field_bytes(self.handle, int(prec), int(Ls)))

    def dwf_import(self, prec, Ls, canon, native):
        _check(self._call(self.lib.lqcd_dwf_import, self.handle, int(prec), int(Ls), _ptr(canon)[0], _ptr(native)[0]),
               "lqcd_dwf_import")

    def dwf_export(self, prec, Ls, native, canon):
        _check(self._call(self.lib.lqcd_dwf_export, self.handle, int(prec), int(Ls), _ptr(native)[0], _ptr(canon)[0]),
               "lqcd_dwf_export")

    def dwf_apply_native_repeat(self, Ls, M5, mf, prec, ins, outs, reps: int, dag=False, b5=1.0, c5=0.0, tmp=None):
        """reps domain-wall applications on native fields, cycling over the (in, out) pairs."""
        d = dwf_params(Ls, M5, mf, b5, c5)
        pi = [_ptr(t)[0] for t in ins]
        po = [_ptr(t)[0] for t in outs]
        pt = _ptr(tmp)[0] if tmp is not None else None
        self._enter()
        try:
            for r in range(int(reps)):
                k = r % len(pi)
                _check(self.lib.lqcd_dwf_apply_native(self.handle, C.byref(d), int(bool(dag)), int(prec), pi[k], po[k],
                                                      pt), "lqcd_dwf_apply_native")
        finally:
            self._exit()

    def stag_field_bytes(self, prec: int) -> int:
        return int(self.lib.lqcd_stag_field_bytes(self.handle, int(prec)))

    def stag_import(self, prec, parity, canon, native):
        _check(self._call(self.lib.lqcd_stag_import, self.handle, int(prec), int(parity), _ptr(canon)[0],
                          _ptr(native)[0]), "lqcd_stag_import")

    def stag_export(self, prec, parity, native, canon):
        _check(self._call(self.lib.lqcd_stag_export, self.handle, int(prec), int(parity), _ptr(native)[0],
                          _ptr(canon)[0]), "lqcd_stag_export")

    def stag_hop_native_repeat(self, prec, out_parity, ins, outs, reps: int):
        """reps launches of the staggered hop on native fields, cycling over the (in, out) pairs."""
        pi = [_ptr(t)[0] for t in ins]
        po = [_ptr(t)[0] for t in outs]
        self._enter()
        try:
            for r in range(int(reps)):
                k = r % len(pi)
                _check(self.lib.lqcd_stag_hop_native(self.handle, int(prec), int(out_parity), pi[k], po[k]),
                       "lqcd_stag_hop_native")
        finally:
            self._exit()

    def stag_solve(self, mass, b, x, tol=1e-10, max_iter=100000, max_outer=20, raise_on_fail=True,
                   inner_prec=F64, inner_tol=0.0) -> Stats:
        """Staggered D x = b by CG on the even-odd normal system (FP64, or FP32
        inner solves under FP64 defect correction with inner_prec=F32)."""
        prm = default_params()
        pb, db = _ptr(b)
        px, dx = _ptr(x)
        if db != dx:
            raise ValueError("b and x must both be host or both be device")
        prm.tol, prm.max_iter, prm.max_outer, prm.on_device = float(tol), int(max_iter), int(max_outer), db
        prm.inner_prec, prm.inner_tol = int(inner_prec), float(inner_tol)
        st = SolveStats()
        status = self._call(self.lib.lqcd_stag_solve, self.handle, float(mass), pb, px, C.byref(prm), C.byref(st))
        if raise_on_fail:
            _check(status, "lqcd_stag_solve")
        return Stats(st.outer_iters, st.inner_iters, st.restarts, st.true_rel_resid, st.seconds_solve,
                     st.seconds_setup, status)


def batch_autotune(lattices, nrhs, prec=F32, shape=None):
    """Launch shapes of the batched hops for these lattices with nrhs[k]
    right-hand sides each (tuned per kind of hop, cached or, with shape =
    (nb, nw, nslot, walk, nt), forced for every kind); returns (shape of the
    A_oo^-1 H_oe hop, microseconds per launch of that hop)."""
    lib = load()
    n = len(lattices)
    ctxs = (C.c_void_p * n)(*[lat.handle.value for lat in lattices])
    nr = (C.c_int * n)(*[int(k) for k in nrhs])
    sh = (C.c_int * 5)(*(tuple(shape) if shape is not None else (0, 0, 0, 0, 0)))
    us = C.c_double(0.0)
    _check(lib.lqcd_batch_autotune(ctxs, nr, n, int(prec), sh, C.byref(us)), "lqcd_batch_autotune")
    return tuple(sh[k] for k in range(5)), us.value


def batch_apply_schur(lattices, ins, outs, prec=F32):
    """outs[k][r] = S ins[k][r] through the batched kernels (device arrays of
    shape [nrhs, Lt, Lz, Ly, Lx, 4, 3])."""
    lib = load()
    n = len(lattices)
    ctxs = (C.c_void_p * n)(*[lat.handle.value for lat in lattices])
    nr = (C.c_int * n)(*[int(b.shape[0]) for b in ins])
    pi = [_ptr(b) for b in ins]
    po = [_ptr(x) for x in outs]
    if any(d != 1 for _, d in pi + po):
        raise ValueError("batch_apply_schur takes device arrays")
    _check(lib.lqcd_batch_apply_schur(ctxs, nr, n, int(prec), (C.c_void_p * n)(*[p for p, _ in pi]),
                                      (C.c_void_p * n)(*[p for p, _ in po])), "lqcd_batch_apply_schur")
    return outs


def solve_batch(lattices, bs, xs, tol=1e-10, inner_prec=F32, inner_tol=0.0, check_every=8, use_graph=True):
    """Batched solve: bs[k] / xs[k] hold nrhs[k] canonical vectors of lattices[k] back to back
    (arrays of shape [nrhs, Lt, Lz, Ly, Lx, 4, 3]); returns one Stats per RHS."""
    lib = load()
    n = len(lattices)
    ctxs = (C.c_void_p * n)(*[lat.handle.value for lat in lattices])
    nrhs = (C.c_int * n)(*[int(b.shape[0]) for b in bs])
    pbs = [_ptr(b) for b in bs]
    pxs = [_ptr(x) for x in xs]
    devs = {d for _, d in pbs + pxs}
    if len(devs) != 1:
        raise ValueError("all b and x must be on the same side")
    prm = default_params()
    prm.tol, prm.inner_prec, prm.inner_tol = float(tol), int(inner_prec), float(inner_tol)
    prm.check_every, prm.use_graph, prm.on_device = int(check_every), int(bool(use_graph)), devs.pop()
    total = sum(int(b.shape[0]) for b in bs)
    st = (SolveStats * total)()
    for lat in lattices:
        lat._enter()
    try:
        status = lib.lqcd_solve_batch(ctxs, nrhs, (C.c_void_p * n)(*[p for p, _ in pbs]),
                                      (C.c_void_p * n)(*[p for p, _ in pxs]), n, C.byref(prm), st)
    finally:
        for lat in lattices:
            lat._exit()
    _check(status, "lqcd_solve_batch")
    return [Stats(s.outer_iters, s.inner_iters, s.restarts, s.true_rel_resid, s.seconds_solve, s.seconds_setup,
                  status) for s in st]
