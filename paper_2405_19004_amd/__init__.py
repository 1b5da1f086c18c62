"""Python binding of the vertex-patch multigrid library (libvps.so, gfx950).

Argument marshalling only: every step runs in the HIP library behind the C-ABI
declared in include/vps.h.  Functions keep the C names (vps_create,
vps_smoother_apply, ...) and take raw device pointers; the `Problem` class adds
shape/dtype checks on torch tensors before any pointer reaches a kernel.  The
library must be built (python -m paper_2405_19004_amd.build); importing the
binding without it raises, there is no fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# VPS_LIB may name another build of the same library (A/B timing of kernel variants).
LIB_PATH = os.environ.get("VPS_LIB") or os.path.join(_HERE, "libvps.so")

VPS_OK, VPS_EINVAL, VPS_ENOMEM, VPS_EHIP, VPS_ENOCONV, VPS_EBREAKDOWN, VPS_ENOTFINITE, VPS_EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
VPS_FP64, VPS_FP32 = 0, 1
VPS_MULTIPLICATIVE, VPS_ADDITIVE, VPS_MULTIPLICATIVE_BOUNDARY, VPS_MULTIPLICATIVE_SEPARATE = 0, 1, 2, 3
VPS_MULTIPLICATIVE_MFMA = 4
VPS_SOLVE_FP64, VPS_SOLVE_MIXED = 0, 1
VPS_FLAG_FP64_HIERARCHY, VPS_FLAG_FP32_HIERARCHY, VPS_FLAG_NO_SOLVER, VPS_FLAG_POST_SAME_ORDER = 0x1, 0x2, 0x4, 0x8
VPS_FLAG_BOUNDARY_SMOOTHER, VPS_FLAG_GRAPHS, VPS_FLAG_SEPARATE_SMOOTHER = 0x10, 0x20, 0x40
VPS_FLAG_MFMA_SMOOTHER = 0x80

_STATUS_NAMES = {0: "VPS_OK", -1: "VPS_EINVAL", -2: "VPS_ENOMEM", -3: "VPS_EHIP", -4: "VPS_ENOCONV",
                 -5: "VPS_EBREAKDOWN", -6: "VPS_ENOTFINITE", -7: "VPS_EBUSY"}


class VpsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (_STATUS_NAMES.get(status, "?"), status, msg))
        self.status = status


class LevelInfo(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("degree", ctypes.c_int), ("level", ctypes.c_int),
                ("n1d", ctypes.c_longlong), ("n_dofs", ctypes.c_longlong), ("n_interior", ctypes.c_longlong),
                ("n_cells", ctypes.c_longlong), ("n_patches", ctypes.c_longlong), ("n_colors", ctypes.c_int),
                ("color_count", ctypes.c_longlong * 8), ("h", ctypes.c_double)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("true_rel_residual", ctypes.c_double), ("status", ctypes.c_int)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_LL = ctypes.c_longlong
_SIGS = {
    "vps_create": (_I, [_I, _I, _I, ctypes.c_uint, _P, ctypes.POINTER(_P)]),
    "vps_destroy": (_I, [_P]),
    "vps_footprint_bytes": (_I, [_I, _I, _I, ctypes.c_uint, ctypes.POINTER(ctypes.c_size_t)]),
    "vps_level_info": (_I, [_P, _I, ctypes.POINTER(LevelInfo)]),
    "vps_dof_index": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_LL)]),
    "vps_patch_first_index": (_I, [_P, _I, _I, ctypes.POINTER(_LL), _LL, ctypes.POINTER(_LL)]),
    "vps_operator_apply": (_I, [_P, _I, _I, _P, _P]),
    "vps_residual": (_I, [_P, _I, _I, _P, _P, _P]),
    "vps_smoother_apply": (_I, [_P, _I, _I, _I, _I, _P, _P]),
    "vps_color_pass": (_I, [_P, _I, _I, _I, _I, _P, _P]),
    "vps_restrict": (_I, [_P, _I, _I, _P, _P]),
    "vps_restrict_noalloc": (_I, [_I, _I, _I, _I, _P, _P, _P]),
    "vps_launch_geometry_check": (_I, [_I, _I, _I, ctypes.POINTER(_LL)]),
    "vps_prolongate_add": (_I, [_P, _I, _I, _P, _P]),
    "vps_coarse_solve": (_I, [_P, _I, _P, _P]),
    "vps_vcycle": (_I, [_P, _I, _P, _P]),
    "vps_pcg_solve": (_I, [_P, _I, _P, _P, ctypes.c_double, _I, ctypes.POINTER(SolveStats)]),
    "vps_rhs_sine_modes": (_I, [_P, _I, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double), _P]),
    "vps_fmg_solve": (_I, [_P, _I, ctypes.POINTER(_P), _P, ctypes.c_double, _I, ctypes.POINTER(SolveStats)]),
    "vps_l2_error_sine_modes": (_I, [_P, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double), _I, _P,
                                     ctypes.POINTER(ctypes.c_double)]),
    "vps_synchronize": (_I, [_P]),
    "vps_last_error": (ctypes.c_char_p, []),
    "vps_host_table": (_I, [_I, _I, ctypes.POINTER(ctypes.c_double), _I, ctypes.POINTER(_I)]),
    "vps_server_create": (_I, [ctypes.c_size_t, _I, _P, ctypes.POINTER(_P)]),
    "vps_server_submit": (_I, [_P, _I, _I, _I, _P, _P, ctypes.c_double, _I, _I, ctypes.POINTER(_LL)]),
    "vps_server_step": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "vps_server_poll": (_I, [_P, _LL, ctypes.POINTER(_I), ctypes.POINTER(SolveStats)]),
    "vps_server_completed": (_I, [_P, ctypes.POINTER(_LL), _I, ctypes.POINTER(_I)]),
    "vps_server_memory": (_I, [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "vps_server_destroy": (_I, [_P]),
    "vps_server_inject_fault": (_I, [_P, _LL, _I]),
}

_lib = None


def lib():
    """Load libvps.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libvps.so is not built: run python -m paper_2405_19004_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def last_error():
    return lib().vps_last_error().decode()


def check(status):
    if status != VPS_OK:
        raise VpsError(status, last_error())
    return status


def _call(name, *args):
    return check(getattr(lib(), name)(*args))


# ----------------------------------------------------------------- C names

def vps_create(dim, degree, fine_level, flags=VPS_FLAG_FP64_HIERARCHY, hip_stream=None):
    h = _P()
    _call("vps_create", dim, degree, fine_level, flags, hip_stream, ctypes.byref(h))
    return h


def vps_destroy(h):
    return _call("vps_destroy", h)


def vps_footprint_bytes(dim, degree, fine_level, flags=VPS_FLAG_FP64_HIERARCHY):
    out = ctypes.c_size_t()
    _call("vps_footprint_bytes", dim, degree, fine_level, flags, ctypes.byref(out))
    return out.value


def vps_level_info(h, level):
    info = LevelInfo()
    _call("vps_level_info", h, level, ctypes.byref(info))
    return info


def vps_dof_index(h, level, coords):
    c = (_I * len(coords))(*coords)
    out = _LL()
    _call("vps_dof_index", h, level, c, ctypes.byref(out))
    return out.value


def vps_patch_first_index(h, level, color):
    n = _LL()
    _call("vps_patch_first_index", h, level, color, None, 0, ctypes.byref(n))
    buf = (_LL * max(n.value, 1))()
    _call("vps_patch_first_index", h, level, color, buf, n.value, ctypes.byref(n))
    return list(buf[:n.value])


def vps_operator_apply(h, level, prec, x_ptr, y_ptr):
    return _call("vps_operator_apply", h, level, prec, x_ptr, y_ptr)


def vps_residual(h, level, prec, b_ptr, x_ptr, r_ptr):
    return _call("vps_residual", h, level, prec, b_ptr, x_ptr, r_ptr)


def vps_smoother_apply(h, level, prec, mode, reverse_colors, b_ptr, x_ptr):
    return _call("vps_smoother_apply", h, level, prec, mode, int(reverse_colors), b_ptr, x_ptr)


def vps_color_pass(h, level, prec, mode, color, b_ptr, x_ptr):
    return _call("vps_color_pass", h, level, prec, mode, color, b_ptr, x_ptr)


def vps_restrict(h, fine_level, prec, rf_ptr, rc_ptr):
    return _call("vps_restrict", h, fine_level, prec, rf_ptr, rc_ptr)


def vps_launch_geometry_check(dim, degree, fine_level):
    """Host-side check of every launch of a hierarchy; returns the colour-pass workgroups checked."""
    n = _LL()
    _call("vps_launch_geometry_check", dim, degree, fine_level, ctypes.byref(n))
    return n.value


def vps_restrict_noalloc(dim, degree, fine_level, prec, rf_ptr, rc_ptr, hip_stream=None):
    return _call("vps_restrict_noalloc", dim, degree, fine_level, prec, rf_ptr, rc_ptr, hip_stream)


def vps_prolongate_add(h, fine_level, prec, e_ptr, x_ptr):
    return _call("vps_prolongate_add", h, fine_level, prec, e_ptr, x_ptr)


def vps_coarse_solve(h, prec, b_ptr, x_ptr):
    return _call("vps_coarse_solve", h, prec, b_ptr, x_ptr)


def vps_vcycle(h, prec, b_ptr, x_ptr):
    return _call("vps_vcycle", h, prec, b_ptr, x_ptr)


def vps_pcg_solve(h, solve_mode, b_ptr, x_ptr, rtol, maxit):
    st = SolveStats()
    status = lib().vps_pcg_solve(h, solve_mode, b_ptr, x_ptr, rtol, maxit, ctypes.byref(st))
    if status not in (VPS_OK, VPS_ENOCONV):
        raise VpsError(status, last_error())
    return st


def vps_fmg_solve(h, prec, b_ptrs, x_ptr, eps, maxit):
    st = SolveStats()
    arr = (_P * len(b_ptrs))(*b_ptrs)
    status = lib().vps_fmg_solve(h, prec, arr, x_ptr, eps, maxit, ctypes.byref(st))
    if status not in (VPS_OK, VPS_ENOCONV):
        raise VpsError(status, last_error())
    return st


def vps_rhs_sine_modes(h, level, prec, kappas, coefs, b_ptr):
    flat = [int(v) for kap in kappas for v in kap]
    kap = (_I * max(len(flat), 1))(*flat)
    co = (ctypes.c_double * max(len(coefs), 1))(*[float(c) for c in coefs])
    return _call("vps_rhs_sine_modes", h, level, prec, len(coefs), kap, co, b_ptr)


def vps_l2_error_sine_modes(h, level, kappas, ucoefs, nq, x_ptr):
    flat = [int(v) for kap in kappas for v in kap]
    kap = (_I * max(len(flat), 1))(*flat)
    co = (ctypes.c_double * max(len(ucoefs), 1))(*[float(c) for c in ucoefs])
    err = ctypes.c_double()
    _call("vps_l2_error_sine_modes", h, level, len(ucoefs), kap, co, nq, x_ptr, ctypes.byref(err))
    return err.value


def vps_synchronize(h):
    return _call("vps_synchronize", h)


def vps_host_table(k, which):
    n = _I()
    _call("vps_host_table", k, which, None, 0, ctypes.byref(n))
    buf = (ctypes.c_double * n.value)()
    _call("vps_host_table", k, which, buf, n.value, ctypes.byref(n))
    return list(buf)


def vps_server_create(budget_bytes, max_active, hip_stream=None):
    """hip_stream: the caller's stream as an integer handle; default torch's current stream."""
    if hip_stream is None:
        import torch
        if torch.cuda.is_available():
            hip_stream = torch.cuda.current_stream().cuda_stream
    h = _P()
    _call("vps_server_create", budget_bytes, max_active, hip_stream, ctypes.byref(h))
    return h


def vps_server_submit(s, dim, degree, level, b_ptr, x_ptr, rtol, solve_mode, maxit):
    t = _LL()
    _call("vps_server_submit", s, dim, degree, level, b_ptr, x_ptr, rtol, solve_mode, maxit, ctypes.byref(t))
    return t.value


def vps_server_step(s):
    a, q = _I(), _I()
    _call("vps_server_step", s, ctypes.byref(a), ctypes.byref(q))
    return a.value, q.value


def vps_server_poll(s, ticket):
    done = _I()
    st = SolveStats()
    _call("vps_server_poll", s, ticket, ctypes.byref(done), ctypes.byref(st))
    return bool(done.value), st


def vps_server_completed(s, cap=4096):
    """Tickets finished since the previous call (completion order)."""
    out = []
    buf = (_LL * cap)()
    n = _I()
    while True:
        _call("vps_server_completed", s, buf, cap, ctypes.byref(n))
        out.extend(buf[i] for i in range(n.value))
        if n.value < cap:
            return out


def vps_server_memory(s):
    a, c = ctypes.c_size_t(), ctypes.c_size_t()
    _call("vps_server_memory", s, ctypes.byref(a), ctypes.byref(c))
    return a.value, c.value


def vps_server_destroy(s):
    return _call("vps_server_destroy", s)


def vps_server_inject_fault(s, ticket, stage):
    return _call("vps_server_inject_fault", s, ticket, stage)


# ------------------------------------------------------------ torch layer

class Problem:
    """One level hierarchy; vectors are contiguous torch tensors on the GPU.

    Every method checks device, dtype, contiguity and length on the host before
    handing pointers to the library, so a kernel never sees a short buffer.
    """

    def __init__(self, dim, degree, fine_level, flags=VPS_FLAG_FP64_HIERARCHY | VPS_FLAG_FP32_HIERARCHY,
                 stream=None):
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("the vertex-patch library needs a ROCm GPU")
        self.dim, self.degree, self.L, self.flags = dim, degree, fine_level, flags
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = vps_create(dim, degree, fine_level, flags, ctypes.c_void_p(self.stream.cuda_stream))

    def close(self):
        if self.h:
            vps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def n1d(self, level=None):
        return self.degree * 2 ** (self.L if level is None else level) + 1

    def n(self, level=None):
        return self.n1d(level) ** self.dim

    def info(self, level=None):
        return vps_level_info(self.h, self.L if level is None else level)

    def _prec(self, t):
        torch = self.torch
        if t.dtype == torch.float64:
            return VPS_FP64
        if t.dtype == torch.float32:
            return VPS_FP32
        raise TypeError("vectors must be float64 or float32")

    def _chk(self, level, *ts):
        prec = self._prec(ts[0])
        for t in ts:
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("vectors must be contiguous GPU tensors")
            if self._prec(t) != prec:
                raise TypeError("all vectors of one call must share a dtype")
            if t.numel() != self.n(level):
                raise ValueError("vector length %d != %d nodes of level %d" % (t.numel(), self.n(level), level))
        return prec

    def new(self, dtype=None, level=None):
        torch = self.torch
        return torch.zeros(self.n(level), dtype=dtype or torch.float64, device="cuda")

    def operator_apply(self, x, y=None, level=None):
        level = self.L if level is None else level
        y = torch_empty_like(x) if y is None else y
        prec = self._chk(level, x, y)
        vps_operator_apply(self.h, level, prec, x.data_ptr(), y.data_ptr())
        return y

    def residual(self, b, x, r=None, level=None):
        level = self.L if level is None else level
        r = torch_empty_like(x) if r is None else r
        prec = self._chk(level, b, x, r)
        vps_residual(self.h, level, prec, b.data_ptr(), x.data_ptr(), r.data_ptr())
        return r

    def smoother_apply(self, b, x, mode=VPS_MULTIPLICATIVE, reverse=False, level=None):
        level = self.L if level is None else level
        prec = self._chk(level, b, x)
        vps_smoother_apply(self.h, level, prec, mode, reverse, b.data_ptr(), x.data_ptr())
        return x

    def color_pass(self, b, x, color, mode=VPS_MULTIPLICATIVE, level=None):
        level = self.L if level is None else level
        prec = self._chk(level, b, x)
        vps_color_pass(self.h, level, prec, mode, color, b.data_ptr(), x.data_ptr())
        return x

    def restrict(self, r_fine, r_coarse=None, fine_level=None):
        fine_level = self.L if fine_level is None else fine_level
        if r_coarse is None:
            r_coarse = self.torch.zeros(self.n(fine_level - 1), dtype=r_fine.dtype, device="cuda")
        prec = self._chk(fine_level, r_fine)
        if self._chk(fine_level - 1, r_coarse) != prec:
            raise TypeError("dtype mismatch")
        vps_restrict(self.h, fine_level, prec, r_fine.data_ptr(), r_coarse.data_ptr())
        return r_coarse

    def prolongate_add(self, e_coarse, x_fine, fine_level=None):
        fine_level = self.L if fine_level is None else fine_level
        prec = self._chk(fine_level, x_fine)
        if self._chk(fine_level - 1, e_coarse) != prec:
            raise TypeError("dtype mismatch")
        vps_prolongate_add(self.h, fine_level, prec, e_coarse.data_ptr(), x_fine.data_ptr())
        return x_fine

    def coarse_solve(self, b, x):
        prec = self._chk(1, b, x)
        vps_coarse_solve(self.h, prec, b.data_ptr(), x.data_ptr())
        return x

    def vcycle(self, b, x):
        prec = self._chk(self.L, b, x)
        vps_vcycle(self.h, prec, b.data_ptr(), x.data_ptr())
        return x

    def pcg_solve(self, b, x=None, rtol=1e-8, maxit=100, mode=VPS_SOLVE_FP64):
        x = self.new() if x is None else x
        if self._chk(self.L, b, x) != VPS_FP64:
            raise TypeError("pcg_solve takes float64 vectors")
        st = vps_pcg_solve(self.h, mode, b.data_ptr(), x.data_ptr(), rtol, maxit)
        return x, st

    def fmg_solve(self, b_levels, x=None, eps=1e-9, maxit=50):
        """Full multigrid; b_levels[l-1] is the right-hand side of level l (l = 1..L), one dtype."""
        if len(b_levels) != self.L:
            raise ValueError("need one right-hand side per level (%d)" % self.L)
        prec = None
        for lvl, b in enumerate(b_levels, start=1):
            p = self._chk(lvl, b)
            if prec is not None and p != prec:
                raise TypeError("all levels must share a dtype")
            prec = p
        x = self.new(b_levels[0].dtype) if x is None else x
        if self._chk(self.L, x) != prec:
            raise TypeError("x must have the right-hand sides' dtype")
        st = vps_fmg_solve(self.h, prec, [b.data_ptr() for b in b_levels], x.data_ptr(), eps, maxit)
        return x, st

    def rhs_sine_modes(self, kappas, coefs, b=None, level=None, dtype=None):
        level = self.L if level is None else level
        b = self.new(dtype, level) if b is None else b
        for kap in kappas:
            if len(kap) != self.dim:
                raise ValueError("each mode needs %d wave numbers" % self.dim)
        prec = self._chk(level, b)
        vps_rhs_sine_modes(self.h, level, prec, kappas, coefs, b.data_ptr())
        return b

    def l2_error_sine_modes(self, x, kappas, ucoefs, level=None, nq=0):
        """L2 error of the FP64 nodal vector x against sum ucoefs[m] prod_a sin(pi kappas[m][a] x_a)."""
        level = self.L if level is None else level
        for kap in kappas:
            if len(kap) != self.dim:
                raise ValueError("each mode needs %d wave numbers" % self.dim)
        prec = self._chk(level, x)
        if prec != VPS_FP64:
            raise ValueError("x must be FP64")
        return vps_l2_error_sine_modes(self.h, level, kappas, ucoefs, nq, x.data_ptr())

    def synchronize(self):
        vps_synchronize(self.h)


def torch_empty_like(t):
    import torch
    return torch.empty_like(t)
