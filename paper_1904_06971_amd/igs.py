"""Thin Python binding of libigs (argument marshalling only).

Every numerical step runs in the HIP kernels behind the C ABI declared in
``include/igs.h``; this module converts problem descriptions to the C structs,
takes device pointers and the current stream from torch tensors, and raises
on error statuses.  There is no CPU fallback: when ``libigs.so`` is missing
the first call raises ``IGSError``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libigs.so")

IGS_OK = 0
STATUS = {0: "IGS_OK", -1: "IGS_ERR_ARG", -2: "IGS_ERR_UNSUPPORTED", -3: "IGS_ERR_KNOTS", -4: "IGS_ERR_SAMPLES",
          -5: "IGS_ERR_GEOMETRY", -6: "IGS_ERR_HIP", -7: "IGS_ERR_NOMEM",
          -8: "IGS_ERR_SCRATCH", 1: "IGS_NOT_CONVERGED", 2: "IGS_BREAKDOWN"}
STIFFNESS, MASS = 0, 1
F64, F32 = 0, 1
GEOM = {"identity": 0, "sine": 1, "poly2": 2}
COEF = {"const": 0, "sine3": 1, "spline": 2, "exp_spline": 3}
SRC_CONST, SRC_SINE = 0, 1
EXPORTS = ["igs_band_layout", "igs_validate", "igs_surrogate_layout", "igs_sampling_length", "igs_status_string",
           "igs_version",
           "igs_assemble_exact", "igs_assemble_surrogate", "igs_assemble_noalloc", "igs_assemble_surrogate_fe",
           "igs_surrogate_fe_layout", "igs_assemble_surrogate_pd", "igs_surrogate_pd_layout", "igs_plan_create",
           "igs_plan_create_fe", "igs_plan_create_pd", "igs_plan_create_mf",
           "igs_apply_mf", "igs_solve_cg_mf", "igs_plan_execute", "igs_plan_destroy",
           "igs_assemble_rhs", "igs_assemble_async", "igs_assemble_rhs_async", "igs_check", "igs_apply", "igs_solve_cg", "igs_apply_vjp", "igs_compliance_grad",
           "igs_profile_enable", "igs_profile_read"]


class IGSError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({_status_text(status)})")


class Geometry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("a", ctypes.c_double)]


class Coef(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("c0", ctypes.c_double), ("amp", ctypes.c_double),
                ("degree", ctypes.c_int32), ("ncoef", ctypes.c_int32 * 3), ("coef", ctypes.c_void_p)]


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("p", ctypes.c_int32), ("nelem", ctypes.c_int32 * 3),
                ("nquad", ctypes.c_int32), ("batch", ctypes.c_int32), ("knots", ctypes.c_void_p * 3),
                ("geom", Geometry), ("coef", Coef)]


class Layout(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32 * 3), ("slots", ctypes.c_int32), ("upper", ctypes.c_int32),
                ("N", ctypes.c_int64), ("ld", ctypes.c_int64), ("band_elems", ctypes.c_int64)]


class SurrogateInfo(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int32 * 3), ("interior", ctypes.c_int32 * 3), ("sample_rows", ctypes.c_int64),
                ("boundary_rows", ctypes.c_int64), ("quadrature_rows", ctypes.c_int64)]


class FEInfo(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int32 * 3), ("classes", ctypes.c_int64), ("corner_rows", ctypes.c_int64),
                ("quadrature_rows", ctypes.c_int64)]


class PDInfo(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int32 * 3), ("max_samples", ctypes.c_int32 * 3),
                ("noncardinal_rows", ctypes.c_int64), ("quadrature_rows", ctypes.c_int64)]


class ProfilePhase(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int32), ("ms", ctypes.c_double)]


class Profile(ctypes.Structure):
    _fields_ = [("nphase", ctypes.c_int32), ("phase", ProfilePhase * 24)]


class CgInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("outer_iterations", ctypes.c_int32), ("status", ctypes.c_int32),
                ("relres", ctypes.c_double)]


_lib = None


def lib():
    """Load libigs.so (built in-tree by paper_1904_06971_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise IGSError(-6, f"libigs.so not found at {LIB_PATH}; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(Problem)
        vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        sigs = {
            "igs_band_layout": [P, ctypes.POINTER(Layout)],
            "igs_validate": [P, i32, i32],
            "igs_surrogate_layout": [P, i32, i32, ctypes.POINTER(SurrogateInfo), ctypes.POINTER(ctypes.c_int32), i32],
            "igs_sampling_length": [i32, i32, i32, f64, f64],
            "igs_assemble_exact": [P, i32, i32, vp, vp],
            "igs_assemble_surrogate": [P, i32, i32, i32, i32, vp, vp],
            "igs_assemble_noalloc": [P, i32, i32, i32, i32, vp, vp],
            "igs_assemble_surrogate_fe": [P, i32, i32, i32, i32, vp, vp],
            "igs_surrogate_fe_layout": [P, i32, i32, ctypes.POINTER(FEInfo)],
            "igs_plan_create_fe": [P, i32, i32, i32, i32, vp, ctypes.POINTER(vp)],
            "igs_assemble_surrogate_pd": [P, i32, i32, i32, i32, vp, vp],
            "igs_surrogate_pd_layout": [P, i32, i32, ctypes.POINTER(PDInfo)],
            "igs_plan_create_pd": [P, i32, i32, i32, i32, vp, ctypes.POINTER(vp)],
            "igs_plan_create_mf": [P, i32, i32, i32, vp, ctypes.POINTER(vp)],
            "igs_apply_mf": [vp, vp, vp, vp, i32, vp],
            "igs_solve_cg_mf": [vp, vp, vp, vp, f64, i32, ctypes.POINTER(CgInfo), vp],
            "igs_plan_create": [P, i32, i32, i32, i32, vp, ctypes.POINTER(vp)],
            "igs_plan_execute": [vp, vp, vp, vp],
            "igs_plan_destroy": [vp],
            "igs_assemble_rhs": [P, i32, f64, vp, vp],
            "igs_assemble_async": [P, i32, i32, i32, i32, vp, vp],
            "igs_assemble_rhs_async": [P, i32, f64, vp, vp],
            "igs_check": [vp],
            "igs_apply": [P, i32, vp, vp, vp, i32, vp],
            "igs_solve_cg": [P, vp, vp, vp, vp, f64, i32, ctypes.POINTER(CgInfo), vp],
            "igs_apply_vjp": [P, i32, i32, vp, vp, vp, vp, vp, vp],
            "igs_compliance_grad": [P, i32, i32, vp, vp, vp],
            "igs_profile_enable": [i32],
            "igs_profile_read": [ctypes.POINTER(Profile)],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int32
        L.igs_status_string.argtypes = [ctypes.c_int32]
        L.igs_status_string.restype = ctypes.c_char_p
        L.igs_version.argtypes = []
        L.igs_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _status_text(st):
    try:
        return lib().igs_status_string(st).decode()
    except Exception:  # library missing
        return ""


def _check(st, where):
    if st != IGS_OK:
        raise IGSError(st, where)


def profile_enable(on=True):
    _check(lib().igs_profile_enable(int(on)), "igs_profile_enable")


def profile_read():
    """{phase name: (launches, summed ms)} of the calls since the last read."""
    pr = Profile()
    _check(lib().igs_profile_read(ctypes.byref(pr)), "igs_profile_read")
    return {pr.phase[k].name.decode(): (pr.phase[k].launches, pr.phase[k].ms) for k in range(pr.nphase)}


def version():
    return lib().igs_version().decode()


def make_problem(prob, coef_ptr=None, knots=None):
    """C struct for a problem dict (see paper_1904_06971_amd.workloads).
    coef_ptr: device pointer of the spline control values [batch, prod cn]."""
    pb = Problem()
    pb.n = prob["n"]
    pb.p = prob["p"]
    for d in range(3):
        pb.nelem[d] = prob["nelem"][d] if d < prob["n"] else 1
    pb.nquad = prob.get("nq", 0)
    pb.batch = prob.get("batch", 1)
    keep = []
    for d in range(3):
        if knots is not None and d < prob["n"] and knots[d] is not None:
            arr = np.ascontiguousarray(knots[d], dtype=np.float64)
            keep.append(arr)
            pb.knots[d] = arr.ctypes.data
        else:
            pb.knots[d] = None
    pb.geom.kind = GEOM[prob.get("geom", "identity")]
    pb.geom.a = prob.get("ga", 0.0)
    pb.coef.kind = COEF[prob.get("coef", "const")]
    pb.coef.c0 = prob.get("c0", 1.0)
    pb.coef.amp = prob.get("camp", 0.0)
    pb.coef.degree = prob.get("cdeg", 0)
    cn = prob.get("cn", (0,) * prob["n"])
    for d in range(3):
        pb.coef.ncoef[d] = cn[d] if d < len(cn) else 1
    pb.coef.coef = coef_ptr
    pb._keep = keep
    return pb


def layout(prob):
    out = Layout()
    _check(lib().igs_band_layout(ctypes.byref(make_problem(prob, coef_ptr=1)), ctypes.byref(out)), "igs_band_layout")
    return out


def surrogate_layout(prob, M, q):
    info = SurrogateInfo()
    buf = (ctypes.c_int32 * 4096)()
    _check(lib().igs_surrogate_layout(ctypes.byref(make_problem(prob, coef_ptr=1)), M, q, ctypes.byref(info), buf,
                                      4096), "igs_surrogate_layout")
    idx, pos = [], 0
    for d in range(prob["n"]):
        idx.append(np.array(buf[pos:pos + info.samples[d]], dtype=np.int64))
        pos += info.samples[d]
    return info, idx


def surrogate_fe_layout(prob, M, q):
    info = FEInfo()
    _check(lib().igs_surrogate_fe_layout(ctypes.byref(make_problem(prob, coef_ptr=1)), M, q, ctypes.byref(info)),
           "igs_surrogate_fe_layout")
    return info


def sampling_length(nelem, p, q, c, beta=0.5):
    """Mesh-dependent sampling length M(h) = max{1, floor(c h^((p-q+beta)/(q+1)))}, h = 1/nelem."""
    M = lib().igs_sampling_length(int(nelem), int(p), int(q), float(c), float(beta))
    if M < 1:
        raise IGSError(M, "igs_sampling_length")
    return M


def validate(prob, M=0, q=0):
    return lib().igs_validate(ctypes.byref(make_problem(prob, coef_ptr=1)), M, q)


# ------------------------------------------------------------ torch side ---
def _torch():
    import torch

    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _coef_tensor(prob, device):
    torch = _torch()
    if prob.get("coef") in ("spline", "exp_spline"):
        cc = prob["cc"]
        if isinstance(cc, torch.Tensor):
            return cc.to(device=device, dtype=torch.float64).contiguous()
        return torch.as_tensor(np.asarray(cc, dtype=np.float64), device=device).contiguous()
    return None


def _dt(dtype):
    torch = _torch()
    return (torch.float64, F64) if dtype in (torch.float64, "f64", F64) else (torch.float32, F32)


def empty_band(prob, dtype, device="cuda"):
    torch = _torch()
    lay = layout(prob)
    tdt, _ = _dt(dtype)
    return torch.empty((prob.get("batch", 1), lay.slots, lay.ld), dtype=tdt, device=device)


def assemble_exact(prob, form=STIFFNESS, dtype=None, out=None, device="cuda"):
    """Band [batch, S, ld] of the exactly assembled matrix."""
    torch = _torch()
    tdt, cdt = _dt(dtype if dtype is not None else torch.float64)
    band = out if out is not None else empty_band(prob, tdt, device)
    cc = _coef_tensor(prob, band.device)
    pb = make_problem(prob, None if cc is None else cc.data_ptr())
    _check(lib().igs_assemble_exact(ctypes.byref(pb), form, cdt, band.data_ptr(), _stream()), "igs_assemble_exact")
    return band


def assemble_surrogate(prob, form=STIFFNESS, M=8, q=3, dtype=None, out=None, device="cuda"):
    torch = _torch()
    tdt, cdt = _dt(dtype if dtype is not None else torch.float64)
    band = out if out is not None else empty_band(prob, tdt, device)
    cc = _coef_tensor(prob, band.device)
    pb = make_problem(prob, None if cc is None else cc.data_ptr())
    _check(lib().igs_assemble_surrogate(ctypes.byref(pb), form, M, q, cdt, band.data_ptr(), _stream()),
           "igs_assemble_surrogate")
    return band


def assemble_surrogate_fe(prob, form=STIFFNESS, M=8, q=3, dtype=None, out=None, device="cuda"):
    """igs_assemble_surrogate_fe: surrogate with face/edge stencil functions."""
    torch = _torch()
    tdt, cdt = _dt(dtype if dtype is not None else torch.float64)
    band = out if out is not None else empty_band(prob, tdt, device)
    cc = _coef_tensor(prob, band.device)
    pb = make_problem(prob, None if cc is None else cc.data_ptr())
    _check(lib().igs_assemble_surrogate_fe(ctypes.byref(pb), form, M, q, cdt, band.data_ptr(), _stream()),
           "igs_assemble_surrogate_fe")
    return band


def assemble_surrogate_pd(prob, form=STIFFNESS, M=8, q=3, dtype=None, out=None, device="cuda"):
    """igs_assemble_surrogate_pd: surrogate with a domain per stencil function."""
    torch = _torch()
    tdt, cdt = _dt(dtype if dtype is not None else torch.float64)
    band = out if out is not None else empty_band(prob, tdt, device)
    cc = _coef_tensor(prob, band.device)
    pb = make_problem(prob, None if cc is None else cc.data_ptr())
    _check(lib().igs_assemble_surrogate_pd(ctypes.byref(pb), form, M, q, cdt, band.data_ptr(), _stream()),
           "igs_assemble_surrogate_pd")
    return band


def surrogate_pd_layout(prob, M, q):
    info = PDInfo()
    _check(lib().igs_surrogate_pd_layout(ctypes.byref(make_problem(prob, coef_ptr=1)), M, q, ctypes.byref(info)),
           "igs_surrogate_pd_layout")
    return info


def assemble_noalloc(prob, form=STIFFNESS, M=0, q=3, dtype=None, out=None, device="cuda"):
    """igs_assemble_noalloc: M = 0 full assembly, M >= 1 surrogate, with the
    library's static scratch instead of device allocations (the band is the
    caller's: pass ``out`` to keep the call free of allocations)."""
    torch = _torch()
    tdt, cdt = _dt(dtype if dtype is not None else torch.float64)
    band = out if out is not None else empty_band(prob, tdt, device)
    cc = _coef_tensor(prob, band.device)
    pb = make_problem(prob, None if cc is None else cc.data_ptr())
    _check(lib().igs_assemble_noalloc(ctypes.byref(pb), form, M, q, cdt, band.data_ptr(), _stream()),
           "igs_assemble_noalloc")
    return band


class Plan:
    """A kept assembly plan (igs_plan_*): M = 0 full assembly, M >= 1 surrogate
    (face_edge=True: igs_plan_create_fe; per_delta=True: igs_plan_create_pd;
    matrix_free=True: igs_plan_create_mf).  execute() queues the assembly on
    torch's current stream; the first call synchronises and checks the
    geometry, later calls only queue."""

    def __init__(self, prob, form=STIFFNESS, M=8, q=3, dtype=None, device="cuda", face_edge=False,
                 matrix_free=False, per_delta=False):
        torch = _torch()
        self.prob = prob
        self.tdt, self.cdt = _dt(dtype if dtype is not None else torch.float64)
        self.device = device
        self._cc = _coef_tensor(prob, device)
        pb = make_problem(prob, None if self._cc is None else self._cc.data_ptr())
        h = ctypes.c_void_p()
        if matrix_free:
            _check(lib().igs_plan_create_mf(ctypes.byref(pb), form, M, q, _stream(), ctypes.byref(h)),
                   "igs_plan_create_mf")
        else:
            name = "igs_plan_create_fe" if face_edge else "igs_plan_create_pd" if per_delta else "igs_plan_create"
            _check(getattr(lib(), name)(ctypes.byref(pb), form, M, q, self.cdt, _stream(), ctypes.byref(h)), name)
        self._h = h

    def execute(self, out=None, coef=None):
        """Assemble into out (a new band if None); coef: new spline control
        values [batch, prod cn] (device tensor), else the creation ones."""
        torch = _torch()
        band = out if out is not None else empty_band(self.prob, self.tdt, self.device)
        cp = None
        if coef is not None:
            coef = coef.to(device=band.device, dtype=torch.float64).contiguous()
            self._cc_keep = coef
            cp = coef.data_ptr()
        _check(lib().igs_plan_execute(self._h, cp, band.data_ptr(), _stream()), "igs_plan_execute")
        return band

    def apply(self, band, x, dirichlet=False, out=None):
        """Matrix-free plans: y = A~ x (igs_apply_mf) with the band of the last
        execute()."""
        y = out if out is not None else _torch().empty_like(x)
        _check(lib().igs_apply_mf(self._h, band.data_ptr(), x.data_ptr(), y.data_ptr(), int(bool(dirichlet)),
                                  _stream()), "igs_apply_mf")
        return y

    def solve_cg(self, band, f, u0=None, rtol=1e-10, maxit=100000, check=True):
        """Matrix-free plans: FP64 CG with igs_apply_mf (igs_solve_cg_mf)."""
        torch = _torch()
        u = torch.zeros_like(f) if u0 is None else u0.clone()
        info = CgInfo()
        st = lib().igs_solve_cg_mf(self._h, band.data_ptr(), f.data_ptr(), u.data_ptr(), rtol, maxit,
                                   ctypes.byref(info), _stream())
        if check and st < 0:
            _check(st, "igs_solve_cg_mf")
        return u, {"iterations": info.iterations, "outer_iterations": info.outer_iterations, "status": info.status,
                   "relres": info.relres}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value is not None:
            _check(lib().igs_plan_destroy(self._h), "igs_plan_destroy")
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def assemble_rhs(prob, source=SRC_CONST, c=1.0, out=None, device="cuda"):
    torch = _torch()
    lay = layout(prob)
    f = out if out is not None else torch.empty((prob.get("batch", 1), lay.N), dtype=torch.float64, device=device)
    cc = _coef_tensor(prob, f.device)
    pb = make_problem(prob, None if cc is None else cc.data_ptr())
    _check(lib().igs_assemble_rhs(ctypes.byref(pb), source, float(c), f.data_ptr(), _stream()), "igs_assemble_rhs")
    return f


def assemble_async(prob, form=STIFFNESS, M=0, q=3, dtype=None, out=None, device="cuda"):
    """igs_assemble_async: M = 0 full assembly, M >= 1 surrogate, queued on
    torch's current stream without synchronising; a geometry fault is reported
    by check().  The coefficient tensor of spline kinds is made on the same
    stream, so torch reuses its memory only after the queued kernels."""
    torch = _torch()
    tdt, cdt = _dt(dtype if dtype is not None else torch.float64)
    band = out if out is not None else empty_band(prob, tdt, device)
    cc = _coef_tensor(prob, band.device)
    pb = make_problem(prob, None if cc is None else cc.data_ptr())
    _check(lib().igs_assemble_async(ctypes.byref(pb), form, M, q, cdt, band.data_ptr(), _stream()),
           "igs_assemble_async")
    return band


def assemble_rhs_async(prob, source=SRC_CONST, c=1.0, out=None, device="cuda"):
    """igs_assemble_rhs_async: the load vector, queued without synchronising."""
    torch = _torch()
    lay = layout(prob)
    f = out if out is not None else torch.empty((prob.get("batch", 1), lay.N), dtype=torch.float64, device=device)
    cc = _coef_tensor(prob, f.device)
    pb = make_problem(prob, None if cc is None else cc.data_ptr())
    _check(lib().igs_assemble_rhs_async(ctypes.byref(pb), source, float(c), f.data_ptr(), _stream()),
           "igs_assemble_rhs_async")
    return f


def check():
    """igs_check on torch's current stream: waits for it, raises IGSError
    (IGS_ERR_GEOMETRY) if an asynchronous call queued on it since the last
    check met a folding geometry, and clears that record."""
    _check(lib().igs_check(_stream()), "igs_check")


def apply(prob, band, x, dirichlet=False, out=None):
    torch = _torch()
    _, cdt = _dt(band.dtype)
    x = x.contiguous()
    y = out if out is not None else torch.empty_like(x)
    pb = make_problem(prob, 1)
    _check(lib().igs_apply(ctypes.byref(pb), cdt, band.data_ptr(), x.data_ptr(), y.data_ptr(), int(dirichlet),
                           _stream()), "igs_apply")
    return y


def solve_cg(prob, band64, f, band32=None, u0=None, rtol=1e-10, maxit=100000, check=True):
    """Returns (u, info dict)."""
    torch = _torch()
    u = u0.clone() if u0 is not None else torch.zeros_like(f)
    info = CgInfo()
    pb = make_problem(prob, 1)
    st = lib().igs_solve_cg(ctypes.byref(pb), band64.data_ptr(), None if band32 is None else band32.data_ptr(),
                            f.contiguous().data_ptr(), u.data_ptr(), float(rtol), int(maxit), ctypes.byref(info),
                            _stream())
    if check and st not in (IGS_OK,):
        raise IGSError(st, "igs_solve_cg")
    return u, {"iterations": info.iterations, "outer_iterations": info.outer_iterations, "status": info.status,
               "relres": info.relres}


def apply_vjp(prob, M, q, band64, x, ybar, want_x=True, want_c=True):
    torch = _torch()
    cc = _coef_tensor(prob, x.device)
    pb = make_problem(prob, None if cc is None else cc.data_ptr())
    xbar = torch.empty_like(x) if want_x else None
    cbar = torch.empty_like(cc) if (want_c and cc is not None) else None
    _check(lib().igs_apply_vjp(ctypes.byref(pb), M, q, None if band64 is None else band64.data_ptr(),
                               x.contiguous().data_ptr(), ybar.contiguous().data_ptr(),
                               None if xbar is None else xbar.data_ptr(), None if cbar is None else cbar.data_ptr(),
                               _stream()), "igs_apply_vjp")
    return xbar, cbar


def compliance_grad(prob, M, q, u):
    torch = _torch()
    cc = _coef_tensor(prob, u.device)
    pb = make_problem(prob, None if cc is None else cc.data_ptr())
    cbar = torch.empty_like(cc)
    _check(lib().igs_compliance_grad(ctypes.byref(pb), M, q, u.contiguous().data_ptr(), cbar.data_ptr(), _stream()),
           "igs_compliance_grad")
    return cbar


def band_rows(band, prob, b=0):
    """[N, S] view (host numpy) of problem b's band, for comparisons."""
    lay = layout(prob)
    return band[b, :, :lay.N].T.double().cpu().numpy()
