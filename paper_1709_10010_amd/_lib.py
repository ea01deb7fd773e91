"""ctypes binding of libpwhip.so: argument marshalling only.

Every function here has the name of the C entry point it wraps and does no
arithmetic of the method: it checks dtypes / devices / shapes of torch
tensors, passes raw pointers and sizes, and turns a non-zero status into
``PwError``.  All device work runs in the library's HIP kernels on the
caller's (torch current) stream.  Importing this module fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libpwhip.so")

PW_OK = 0
PW_NOT_CONVERGED = 1
PW_FP64, PW_MIXED_FP32, PW_MIXED_BF16 = 0, 1, 2
PW_TERM_KINETIC, PW_TERM_LOCAL, PW_TERM_NONLOCAL, PW_TERM_EXX, PW_TERM_ALL = 1, 2, 4, 8, 15
PW_PRECOND_NONE, PW_PRECOND_TPA, PW_PRECOND_MLP = 0, 1, 2
PW_PLANE_REGISTER, PW_PLANE_WAVE, PW_PLANE_LDS = 0, 1, 2
STATUS_NAMES = {0: "PW_OK", 1: "PW_NOT_CONVERGED", -1: "PW_ERR_INVALID", -2: "PW_ERR_SHAPE",
                -3: "PW_ERR_NOMEM", -4: "PW_ERR_HIP", -5: "PW_ERR_NOT_FINITE",
                -6: "PW_ERR_NUMERIC"}


class PwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Desc(C.Structure):
    _fields_ = [
        ("cell", C.c_double * 9),
        ("kpt", C.c_double * 3),
        ("ecut", C.c_double),
        ("nr", C.c_int32 * 3),
        ("precision", C.c_int32),
        ("npw", C.c_int64),
        ("miller", C.POINTER(C.c_int32)),
        ("vloc", C.c_void_p),
        ("nproj", C.c_int64),
        ("natom", C.c_int32),
        ("proj_offset", C.POINTER(C.c_int32)),
        ("dij", C.POINTER(C.c_double)),
        ("beta", C.c_void_p),
        ("ld_beta", C.c_int64),
        ("qij", C.POINTER(C.c_double)),
    ]


def _load():
    # torch ships its own HIP runtime with the same soname (libamdhip64.so.7);
    # loading torch first makes the library bind to that one, so the process
    # holds a single HIP runtime whichever module the caller imports first
    import torch  # noqa: F401
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no fallback path")
    lib = C.CDLL(LIBPATH)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "pw_last_error": (C.c_char_p, []),
        "pw_version": (C.c_char_p, []),
        "pw_gsphere": (i32, [C.POINTER(f64), C.POINTER(f64), f64, C.POINTER(i32), i64, C.POINTER(i64)]),
        "pw_workspace_size": (i32, [C.POINTER(_Desc), i64, C.POINTER(C.c_size_t)]),
        "pw_problem_create": (i32, [C.POINTER(_Desc), i64, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "pw_problem_destroy": (i32, [vp]),
        "pw_problem_info": (i32, [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]),
        "pw_hpsi": (i32, [vp, vp, i64, vp, i64, i64, i32, vp]),
        "pw_projections": (i32, [vp, vp, i64, vp, i64, vp]),
        "pw_spsi": (i32, [vp, vp, i64, vp, i64, i64, vp]),
        "pw_precond": (i32, [vp, i32, vp, vp, vp, vp, i64, i64, vp, vp]),
        "pw_davidson_workspace_size": (i32, [vp, i64, i64, C.POINTER(C.c_size_t)]),
        "pw_davidson_create": (i32, [vp, i64, i64, f64, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "pw_davidson_destroy": (i32, [vp]),
        "pw_davidson_init": (i32, [vp, vp, i64, vp]),
        "pw_davidson_step": (i32, [vp, i32, vp, vp, C.POINTER(i32)]),
        "pw_davidson_run": (i32, [vp, i32, i32, vp, vp, C.POINTER(i32)]),
        "pw_davidson_query": (i32, [vp, C.POINTER(f64), C.POINTER(f64), C.POINTER(i32),
                                    C.POINTER(i64), vp]),
        "pw_davidson_vectors": (i32, [vp, vp, i64, vp]),
        "pw_davidson_set_problem": (i32, [vp, vp, vp]),
        "pw_davidson_set_tol": (i32, [vp, f64]),
        "pw_davidson_snapshot": (i32, [vp, vp, vp, vp, vp, i64, vp]),
        "pw_mlp_num_params": (i32, []),
        "pw_mlp_create": (i32, [vp, vp, C.POINTER(vp)]),
        "pw_mlp_destroy": (i32, [vp]),
        "pw_mlp_get": (i32, [vp, vp, vp, vp]),
        "pw_mlp_set": (i32, [vp, vp, vp]),
        "pw_mlp_features": (i32, [vp, vp, vp, vp, vp, i64, i64, vp, vp]),
        "pw_mlp_fit_scaler": (i32, [vp, vp, i64, vp]),
        "pw_mlp_forward": (i32, [vp, vp, i64, vp, vp]),
        "pw_mlp_train_step": (i32, [vp, vp, vp, vp, vp, vp, i64, i64, vp, C.c_float, i32,
                                    C.POINTER(f64), vp]),
        "pw_mlp_targets": (i32, [vp, vp, vp, vp, i64, i64, vp, vp, vp]),
        "pw_batch_create": (i32, [C.POINTER(vp), i32, C.POINTER(vp), C.POINTER(i64), C.POINTER(vp),
                                  C.POINTER(i64), C.POINTER(i64), C.POINTER(vp)]),
        "pw_batch_destroy": (i32, [vp]),
        "pw_batch_hpsi": (i32, [vp, vp]),
        "pw_batch_capture": (i32, [vp, vp]),
        "pw_batch_launch": (i32, [vp, vp]),
        "pw_batch_set_streams": (i32, [vp, C.POINTER(vp), i32]),
        "pw_batch_davidson_create": (i32, [C.POINTER(vp), i32, C.POINTER(vp), i32, C.POINTER(vp)]),
        "pw_batch_davidson_destroy": (i32, [vp]),
        "pw_batch_davidson_init": (i32, [vp, C.POINTER(vp), C.POINTER(i64)]),
        "pw_batch_davidson_step": (i32, [vp, i32, vp, C.POINTER(i32)]),
        "pw_batch_davidson_run": (i32, [vp, C.POINTER(vp), C.POINTER(i64), i32, i32, vp, C.POINTER(i32)]),
        "pw_problem_autotune": (i32, [vp, i64, i32, vp, C.c_size_t, vp, C.POINTER(f64)]),
        "pw_problem_tuning": (i32, [vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(i32), C.POINTER(i32)]),
        "pw_problem_set_tuning": (i32, [vp, i32, i64, i32, i32]),
        "pw_eigh_workspace": (i32, [i32, C.POINTER(C.c_size_t)]),
        "pw_eigh": (i32, [vp, i64, i32, vp, vp, i64, vp, C.c_size_t, vp]),
        "pw_lanczos_workspace_size": (i32, [vp, i64, i32, C.POINTER(C.c_size_t)]),
        "pw_lanczos_create": (i32, [vp, i64, i32, vp, C.c_size_t, C.POINTER(vp)]),
        "pw_lanczos_destroy": (i32, [vp]),
        "pw_lanczos_start": (i32, [vp, vp, i64, vp]),
        "pw_lanczos_run": (i32, [vp, i32, vp]),
        "pw_lanczos_coefficients": (i32, [vp, vp, vp, C.POINTER(i32), vp]),
        "pw_lanczos_resolvent": (i32, [vp, vp, i32, vp, vp]),
        "pw_density_workspace_size": (i32, [vp, C.POINTER(C.c_size_t)]),
        "pw_density": (i32, [vp, vp, i64, i64, C.POINTER(f64), vp, vp, C.c_size_t, vp]),
        "pw_hxc_workspace_size": (i32, [vp, C.POINTER(C.c_size_t)]),
        "pw_hxc": (i32, [vp, vp, vp, vp, C.POINTER(f64), vp, C.c_size_t, vp]),
        "pw_problem_set_vloc": (i32, [vp, vp, vp]),
        "pw_scf_workspace_size": (i32, [vp, C.POINTER(C.c_size_t)]),
        "pw_scf_create": (i32, [vp, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "pw_scf_destroy": (i32, [vp]),
        "pw_scf_step": (i32, [vp, f64, i32, f64, C.POINTER(f64), C.POINTER(i32)]),
        "pw_scf_density": (i32, [vp, vp, vp, vp]),
        "pw_scf_potential": (i32, [vp, vp, vp]),
        "pw_vx_workspace_size": (i32, [vp, i64, C.POINTER(C.c_size_t)]),
        "pw_vx": (i32, [vp, vp, i64, i64, C.POINTER(f64), vp, i64, i64, vp, i64, vp, C.c_size_t, vp]),
        "pw_ace_workspace_size": (i32, [vp, i64, C.POINTER(C.c_size_t)]),
        "pw_ace_set": (i32, [vp, vp, i64, i64, C.POINTER(f64), f64, vp, i64, vp, vp, C.c_size_t, vp]),
        "pw_ace_clear": (i32, [vp]),
        "pw_vx_attach": (i32, [vp, vp, i64, i64, C.POINTER(f64), f64, vp, C.c_size_t, vp]),
        "pw_profile_enable": (i32, [vp, i32]),
        "pw_profile_read": (i32, [vp, C.POINTER(f64), C.POINTER(i64), i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def _check(status: int) -> int:
    if status < 0:
        raise PwError(status, LIB.pw_last_error().decode())
    return status


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a torch tensor on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def _band_block(t, name, npw):
    """(ptr, ld, nbands) of a [nbands][ld] complex128 tensor with unit stride along G."""
    import torch
    ptr = _dev_ptr(t, torch.complex128, name)
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name}: expected a 2-D band-major block with unit stride along G")
    ld = t.stride(0) if t.shape[0] > 1 else max(t.shape[1], npw)
    if t.shape[1] < npw:
        raise ValueError(f"{name}: second dimension {t.shape[1]} < npw {npw}")
    return ptr, int(ld), int(t.shape[0])


def pw_version() -> str:
    return LIB.pw_version().decode()


def pw_gsphere(cell, kpt, ecut: float) -> np.ndarray:
    """Miller triples of {G : |k+G|^2/2 < ecut} in the library's canonical order."""
    cell = np.ascontiguousarray(cell, dtype=np.float64).reshape(9)
    kpt = np.ascontiguousarray(kpt, dtype=np.float64).reshape(3)
    n = C.c_int64(0)
    dp = C.POINTER(C.c_double)
    _check(LIB.pw_gsphere(cell.ctypes.data_as(dp), kpt.ctypes.data_as(dp), float(ecut), None, 0,
                          C.byref(n)))
    out = np.zeros((n.value, 3), dtype=np.int32)
    _check(LIB.pw_gsphere(cell.ctypes.data_as(dp), kpt.ctypes.data_as(dp), float(ecut),
                          out.ctypes.data_as(C.POINTER(C.c_int32)), n.value, C.byref(n)))
    return out


def _workspace(nbytes, device=None):
    """Caller-owned device workspace of nbytes (torch allocations are 256-byte aligned)."""
    import torch
    ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8,
                     device=device if device is not None else "cuda")
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace allocation is not 256-byte aligned")
    return ws


class Problem:
    """Owner of a pw_problem handle and of the workspace bound to it (the
    handle is destroyed before the workspace is released)."""

    def __init__(self, handle, npw, nproj, max_bands, precision, workspace=None):
        self._h = handle
        self.nr = None
        self.npw = npw
        self.nproj = nproj
        self.max_bands = max_bands
        self.precision = precision
        self.workspace = workspace

    @property
    def handle(self):
        if not self._h:
            raise PwError(-1, "problem handle already destroyed")
        return self._h

    def info(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(LIB.pw_problem_info(self.handle, C.byref(a), C.byref(b), C.byref(c)))
        return dict(npw=a.value, nsticks=b.value, nproj=c.value)

    def close(self):
        if self._h:
            LIB.pw_problem_destroy(self._h)
            self._h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pw_problem_create(cell, kpt, ecut, nr, miller, vloc, beta, proj_offset, dij,
                      precision=PW_FP64, max_bands=1, stream=None, qij=None) -> Problem:
    """Wrap pw_problem_create.  vloc: cuda float64 [N0][N1][N2]; beta: cuda complex128
    [nproj][ld] (or None with nproj = 0); miller / proj_offset / dij / qij (overlap
    augmentation in the layout of dij, None for S = 1): host arrays."""
    import torch
    miller = np.ascontiguousarray(miller, dtype=np.int32).reshape(-1, 3)
    d = _Desc()
    d.cell[:] = [float(x) for x in np.asarray(cell, dtype=np.float64).reshape(9)]
    d.kpt[:] = [float(x) for x in np.asarray(kpt, dtype=np.float64).reshape(3)]
    d.ecut = float(ecut)
    d.nr[:] = [int(x) for x in nr]
    d.precision = int(precision)
    d.npw = miller.shape[0]
    d.miller = miller.ctypes.data_as(C.POINTER(C.c_int32))
    if tuple(vloc.shape) != tuple(int(x) for x in nr):
        raise ValueError("vloc shape must equal the grid")
    vloc_c = vloc.contiguous()
    d.vloc = _dev_ptr(vloc_c, torch.float64, "vloc")
    keep = [miller, vloc_c]
    if beta is not None and beta.shape[0] > 0:
        po = np.ascontiguousarray(proj_offset, dtype=np.int32)
        dj = np.ascontiguousarray(dij, dtype=np.float64)
        if beta.stride(1) != 1:
            raise ValueError("beta must have unit stride along G")
        d.nproj = int(beta.shape[0])
        d.natom = int(po.shape[0] - 1)
        d.proj_offset = po.ctypes.data_as(C.POINTER(C.c_int32))
        d.dij = dj.ctypes.data_as(C.POINTER(C.c_double))
        d.beta = _dev_ptr(beta, torch.complex128, "beta")
        d.ld_beta = int(beta.stride(0)) if beta.shape[0] > 1 else int(beta.shape[1])
        keep += [po, dj, beta]
        if qij is not None:
            qj = np.ascontiguousarray(qij, dtype=np.float64)
            if qj.shape != dj.shape:
                raise ValueError("qij must have the layout of dij")
            d.qij = qj.ctypes.data_as(C.POINTER(C.c_double))
            keep.append(qj)
    nbytes = C.c_size_t(0)
    _check(LIB.pw_workspace_size(C.byref(d), int(max_bands), C.byref(nbytes)))
    ws = _workspace(nbytes.value, vloc_c.device)
    h = C.c_void_p()
    _check(LIB.pw_problem_create(C.byref(d), int(max_bands), C.c_void_p(ws.data_ptr()), nbytes.value,
                                 _stream(stream), C.byref(h)))
    del keep
    prob = Problem(h, int(d.npw), int(d.nproj), int(max_bands), int(precision), ws)
    prob.nr = tuple(int(x) for x in nr)
    return prob


def pw_hpsi(prob: Problem, psi, hpsi, terms: int = PW_TERM_ALL, stream=None) -> None:
    ps, ldp, nb = _band_block(psi, "psi", prob.npw)
    hs, ldh, nbh = _band_block(hpsi, "hpsi", prob.npw)
    if nbh < nb:
        raise ValueError("hpsi has fewer bands than psi")
    _check(LIB.pw_hpsi(prob.handle, ps, ldp, hs, ldh, nb, int(terms), _stream(stream)))


def pw_spsi(prob: Problem, psi, spsi, stream=None) -> None:
    ps, ldp, nb = _band_block(psi, "psi", prob.npw)
    ss, lds, nbs = _band_block(spsi, "spsi", prob.npw)
    if nbs < nb:
        raise ValueError("spsi has fewer bands than psi")
    _check(LIB.pw_spsi(prob.handle, ps, ldp, ss, lds, nb, _stream(stream)))


def pw_projections(prob: Problem, psi, proj, stream=None) -> None:
    import torch
    ps, ldp, nb = _band_block(psi, "psi", prob.npw)
    pp = _dev_ptr(proj, torch.complex128, "proj")
    if not proj.is_contiguous() or tuple(proj.shape) != (nb, prob.nproj):
        raise ValueError("proj must be a contiguous [nbands][nproj] tensor")
    _check(LIB.pw_projections(prob.handle, ps, ldp, pp, nb, _stream(stream)))


def pw_precond(prob: Problem, kind: int, theta, x, r, t, net=None, stream=None) -> None:
    import torch
    xs, ldx, nb = _band_block(x, "x", prob.npw)
    rs, ldr, nbr = _band_block(r, "r", prob.npw)
    ts, ldt, nbt = _band_block(t, "t", prob.npw)
    if not (ldx == ldr == ldt) or nbr < nb or nbt < nb:
        raise ValueError("x, r, t must share one leading dimension and band count")
    th = _dev_ptr(theta, torch.float64, "theta") if theta is not None else None
    nh = net.handle if net is not None else None
    _check(LIB.pw_precond(prob.handle, int(kind), th, xs, rs, ts, ldx, nb, nh, _stream(stream)))


PW_NSTAGES = 16
STAGES = ["zfft_inv", "plane", "zfft_fwd", "kinetic", "proj", "dmat", "nlupd", "precond",
          "subgemm", "updgemm", "eig", "chol", "vec", "exx"]


def pw_profile_enable(prob: Problem, on: bool = True) -> None:
    _check(LIB.pw_profile_enable(prob.handle, 1 if on else 0))


def pw_profile_read(prob: Problem, reset: bool = True) -> dict:
    """{stage: (total_ms, launches)} for stages with at least one launch."""
    ms = (C.c_double * PW_NSTAGES)()
    n = (C.c_int64 * PW_NSTAGES)()
    _check(LIB.pw_profile_read(prob.handle, ms, n, 1 if reset else 0))
    return {STAGES[i]: (ms[i], n[i]) for i in range(len(STAGES)) if n[i] > 0}


class Davidson:
    """Owner of a pw_davidson handle and of its workspace."""

    def __init__(self, prob: Problem, nbands: int, max_subspace: int = 0, tol: float = 5e-9,
                 stream=None):
        nbytes = C.c_size_t(0)
        _check(LIB.pw_davidson_workspace_size(prob.handle, int(nbands), int(max_subspace),
                                              C.byref(nbytes)))
        self.workspace = _workspace(nbytes.value)
        h = C.c_void_p()
        _check(LIB.pw_davidson_create(prob.handle, int(nbands), int(max_subspace), float(tol),
                                      C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                      _stream(stream), C.byref(h)))
        self._h = h
        self.prob = prob
        self.nbands = int(nbands)

    @property
    def handle(self):
        if not self._h:
            raise PwError(-1, "Davidson handle already destroyed")
        return self._h

    def close(self):
        if self._h:
            LIB.pw_davidson_destroy(self._h)
            self._h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pw_davidson_init(d: Davidson, psi0, stream=None) -> None:
    ps, ld, nb = _band_block(psi0, "psi0", d.prob.npw)
    if nb < d.nbands:
        raise ValueError("psi0 has fewer bands than the solver")
    _check(LIB.pw_davidson_init(d.handle, ps, ld, _stream(stream)))


def pw_davidson_step(d: Davidson, precond: int = PW_PRECOND_TPA, net=None, stream=None) -> bool:
    c = C.c_int32(0)
    _check(LIB.pw_davidson_step(d.handle, int(precond), net.handle if net is not None else None,
                                _stream(stream), C.byref(c)))
    return bool(c.value)


def pw_davidson_run(d: Davidson, max_iter: int = 200, precond: int = PW_PRECOND_TPA, net=None,
                    stream=None) -> bool:
    c = C.c_int32(0)
    _check(LIB.pw_davidson_run(d.handle, int(max_iter), int(precond),
                               net.handle if net is not None else None, _stream(stream), C.byref(c)))
    return bool(c.value)


def pw_davidson_query(d: Davidson, stream=None) -> dict:
    th = np.zeros(d.nbands)
    rh = np.zeros(d.nbands)
    it = C.c_int32()
    nh = C.c_int64()
    dp = C.POINTER(C.c_double)
    _check(LIB.pw_davidson_query(d.handle, th.ctypes.data_as(dp), rh.ctypes.data_as(dp),
                                 C.byref(it), C.byref(nh), _stream(stream)))
    return dict(theta=th, rho=rh, iterations=it.value, n_hpsi=nh.value)


def pw_davidson_vectors(d: Davidson, x, stream=None) -> None:
    ps, ld, nb = _band_block(x, "x", d.prob.npw)
    if nb < d.nbands:
        raise ValueError("x has fewer bands than the solver")
    _check(LIB.pw_davidson_vectors(d.handle, ps, ld, _stream(stream)))


def pw_davidson_set_tol(d: Davidson, tol: float) -> None:
    _check(LIB.pw_davidson_set_tol(d.handle, float(tol)))


def pw_davidson_set_problem(d: Davidson, prob: Problem, stream=None) -> None:
    _check(LIB.pw_davidson_set_problem(d.handle, prob.handle, _stream(stream)))
    d.prob = prob


def davidson_solve(prob: Problem, psi0, tol: float = 5e-9, max_subspace: int = 0,
                   max_iter: int = 200, precond: int = PW_PRECOND_TPA, net=None,
                   want_vectors: bool = False, refine: Problem = None, refine_tol: float = None,
                   stream=None) -> dict:
    """create + init + run + query (+ vectors) on one problem.

    With ``refine``: run on ``prob`` down to ``tol``, then switch the solve to
    ``refine`` (same sphere, e.g. the FP64 form) and run down to ``refine_tol``.
    """
    import torch
    nb = int(psi0.shape[0])
    d = Davidson(prob, nb, max_subspace, tol, stream)
    try:
        pw_davidson_init(d, psi0, stream)
        conv = pw_davidson_run(d, max_iter, precond, net, stream)
        out = pw_davidson_query(d, stream)
        if refine is not None:
            first = out["iterations"]
            pw_davidson_set_problem(d, refine, stream)
            pw_davidson_set_tol(d, refine_tol if refine_tol else tol)
            conv = pw_davidson_run(d, max_iter, precond, net, stream)
            out = dict(pw_davidson_query(d, stream), iterations_first=first)
        out["converged"] = conv
        if want_vectors:
            x = torch.zeros_like(psi0)
            pw_davidson_vectors(d, x, stream)
            torch.cuda.synchronize()
            out["X"] = x
    finally:
        d.close()
    return out


def pw_davidson_snapshot(d: Davidson, x=None, r=None, theta=None, rho=None, stream=None) -> None:
    """Copies of the last step's Ritz vectors / residuals / values / norms (device tensors)."""
    import torch
    ld = None
    ptrs = []
    for t, name in ((x, "x"), (r, "r")):
        if t is None:
            ptrs.append(None)
        else:
            p_, ld_, nb_ = _band_block(t, name, d.prob.npw)
            if ld is not None and ld_ != ld:
                raise ValueError("x and r must share one leading dimension")
            ld = ld_
            ptrs.append(p_)
    th = _dev_ptr(theta, torch.float64, "theta") if theta is not None else None
    rh = _dev_ptr(rho, torch.float64, "rho") if rho is not None else None
    _check(LIB.pw_davidson_snapshot(d.handle, ptrs[0], ptrs[1], th, rh, ld or d.prob.npw,
                                    _stream(stream)))


MLP_NPARAM = int(LIB.pw_mlp_num_params())


def pack_params(p: dict) -> np.ndarray:
    """Packed float32 parameter vector (W1, b1, W2, b2, W3, b3) from a dict of arrays."""
    return np.concatenate([np.asarray(p[k], dtype=np.float32).reshape(-1)
                           for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def unpack_params(v: np.ndarray) -> dict:
    v = np.asarray(v, dtype=np.float64)
    shapes = (("W1", (64, 4)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (1, 64)),
              ("b3", (1,)))
    out, o = {}, 0
    for k, shp in shapes:
        n = int(np.prod(shp))
        out[k] = v[o:o + n].reshape(shp).copy()
        o += n
    return out


class Mlp:
    """Owner of a pw_mlp handle (FP32 network on the GPU)."""

    def __init__(self, params=None, scaler=None):
        h = C.c_void_p()
        pv = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        sv = None if scaler is None else np.ascontiguousarray(scaler, dtype=np.float32)
        if pv is not None and pv.size != MLP_NPARAM:
            raise ValueError("params must hold pw_mlp_num_params() floats")
        _check(LIB.pw_mlp_create(None if pv is None else pv.ctypes.data_as(C.c_void_p),
                                 None if sv is None else sv.ctypes.data_as(C.c_void_p), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        if not self._h:
            raise PwError(-1, "network handle already destroyed")
        return self._h

    def get(self):
        p = np.zeros(MLP_NPARAM, dtype=np.float32)
        s = np.zeros(8, dtype=np.float32)
        g = np.zeros(MLP_NPARAM, dtype=np.float32)
        _check(LIB.pw_mlp_get(self.handle, p.ctypes.data_as(C.c_void_p), s.ctypes.data_as(C.c_void_p),
                              g.ctypes.data_as(C.c_void_p)))
        return p, s, g

    def set(self, params=None, scaler=None):
        pv = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        sv = None if scaler is None else np.ascontiguousarray(scaler, dtype=np.float32)
        _check(LIB.pw_mlp_set(self.handle, None if pv is None else pv.ctypes.data_as(C.c_void_p),
                              None if sv is None else sv.ctypes.data_as(C.c_void_p)))

    def close(self):
        if self._h:
            LIB.pw_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pw_mlp_features(prob: Problem, theta, x, r, rnorm, F, stream=None) -> None:
    import torch
    rp, ld, nb = _band_block(r, "r", prob.npw)
    xp, ldx, nbx = _band_block(x, "x", prob.npw)
    if ldx != ld or nbx != nb:
        raise ValueError("x and r must have the same shape")
    if F.dtype != torch.float32 or F.numel() < 4 * nb * prob.npw:
        raise ValueError("F must be float32 with room for nbands*npw*4 values")
    _check(LIB.pw_mlp_features(prob.handle, _dev_ptr(theta, torch.float64, "theta"), xp, rp,
                               _dev_ptr(rnorm, torch.float64, "rnorm"), ld, nb,
                               _dev_ptr(F, torch.float32, "F"), _stream(stream)))


def pw_mlp_fit_scaler(net: Mlp, F, stream=None) -> None:
    import torch
    _check(LIB.pw_mlp_fit_scaler(net.handle, _dev_ptr(F, torch.float32, "F"), F.numel() // 4,
                                 _stream(stream)))


def pw_mlp_forward(net: Mlp, F, s, stream=None) -> None:
    import torch
    n = F.numel() // 4
    if s.numel() < n:
        raise ValueError("s too small")
    _check(LIB.pw_mlp_forward(net.handle, _dev_ptr(F, torch.float32, "F"), n,
                              _dev_ptr(s, torch.float32, "s"), _stream(stream)))


def pw_mlp_train_step(net: Mlp, F, R, D, band_off, band_of, s_work, lr=1e-3, update=True,
                      want_loss=True, stream=None):
    import torch
    n = F.numel() // 4
    nb = band_off.numel() - 1
    loss = C.c_double(0.0)
    _check(LIB.pw_mlp_train_step(net.handle, _dev_ptr(F, torch.float32, "F"),
                                 _dev_ptr(R, torch.complex128, "R"), _dev_ptr(D, torch.complex128, "D"),
                                 _dev_ptr(band_off, torch.int64, "band_off"),
                                 _dev_ptr(band_of, torch.int32, "band_of"), nb, n,
                                 _dev_ptr(s_work, torch.float32, "s_work"), float(lr),
                                 1 if update else 0, C.byref(loss) if want_loss else None,
                                 _stream(stream)))
    return loss.value if want_loss else None


def pw_mlp_targets(prob: Problem, Xc, cluster, Xit, D, work, stream=None) -> None:
    import torch
    xp, ld, nb = _band_block(Xc, "Xc", prob.npw)
    ip, ld2, nb2 = _band_block(Xit, "Xit", prob.npw)
    dp, ld3, nb3 = _band_block(D, "D", prob.npw)
    if not (ld == ld2 == ld3 and nb == nb2 == nb3):
        raise ValueError("Xc, Xit, D must share shape")
    if work.numel() < 17 * nb * nb:
        raise ValueError("work must hold 17*nbands^2 complex128")
    _check(LIB.pw_mlp_targets(prob.handle, xp, _dev_ptr(cluster, torch.int32, "cluster"), ip, ld, nb,
                              dp, _dev_ptr(work, torch.complex128, "work"), _stream(stream)))


class Batch:
    """Owner of a pw_batch: problems with their input / output band blocks."""

    def __init__(self, probs, psis, hpsis):
        n = len(probs)
        if not (n == len(psis) == len(hpsis)) or n == 0:
            raise ValueError("one psi and one hpsi block per problem")
        ph = (C.c_void_p * n)(*[p.handle for p in probs])
        xs, ys = (C.c_void_p * n)(), (C.c_void_p * n)()
        lx, ly, nb = (C.c_int64 * n)(), (C.c_int64 * n)(), (C.c_int64 * n)()
        for i, (p, x, y) in enumerate(zip(probs, psis, hpsis)):
            xp, ldx, nbx = _band_block(x, "psi", p.npw)
            yp, ldy, nby = _band_block(y, "hpsi", p.npw)
            if nby < nbx:
                raise ValueError("hpsi has fewer bands than psi")
            xs[i], ys[i], lx[i], ly[i], nb[i] = xp.value, yp.value, ldx, ldy, nbx
        h = C.c_void_p()
        _check(LIB.pw_batch_create(ph, n, xs, lx, ys, ly, nb, C.byref(h)))
        self._h = h
        self._keep = (list(probs), list(psis), list(hpsis))

    @property
    def handle(self):
        if not self._h:
            raise PwError(-1, "batch already destroyed")
        return self._h

    def close(self):
        if self._h:
            LIB.pw_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pw_batch_hpsi(b: Batch, stream=None) -> None:
    _check(LIB.pw_batch_hpsi(b.handle, _stream(stream)))


def pw_batch_capture(b: Batch, stream) -> None:
    _check(LIB.pw_batch_capture(b.handle, _stream(stream)))


def pw_batch_launch(b: Batch, stream=None) -> None:
    _check(LIB.pw_batch_launch(b.handle, _stream(stream)))


def pw_batch_set_streams(b: Batch, streams) -> None:
    """Side streams (torch.cuda.Stream list) for the batch's sweeps; [] restores in-order."""
    n = len(streams)
    arr = (C.c_void_p * max(n, 1))(*[s.cuda_stream for s in streams])
    _check(LIB.pw_batch_set_streams(b.handle, arr, n))
    b._streams = list(streams)


class BatchDavidson:
    """Owner of a pw_batch_dav over Davidson objects (kept alive with it) and
    the torch streams its workers run on."""

    def __init__(self, solvers, streams):
        n, k = len(solvers), len(streams)
        ds = (C.c_void_p * n)(*[d.handle for d in solvers])
        ss = (C.c_void_p * k)(*[s.cuda_stream for s in streams])
        h = C.c_void_p()
        _check(LIB.pw_batch_davidson_create(ds, n, ss, k, C.byref(h)))
        self._h = h
        self.solvers = list(solvers)
        self.streams = list(streams)

    @property
    def handle(self):
        if not self._h:
            raise PwError(-1, "batched Davidson already destroyed")
        return self._h

    def _blocks(self, psi0s):
        n = len(self.solvers)
        if len(psi0s) != n:
            raise ValueError("one start block per solve")
        ptrs, lds = (C.c_void_p * n)(), (C.c_int64 * n)()
        for i, (d, x) in enumerate(zip(self.solvers, psi0s)):
            p_, ld_, nb_ = _band_block(x, "psi0", d.prob.npw)
            if nb_ < d.nbands:
                raise ValueError("psi0 has fewer bands than its solver")
            ptrs[i], lds[i] = p_.value, ld_
        return ptrs, lds

    def init(self, psi0s) -> None:
        ptrs, lds = self._blocks(psi0s)
        _check(LIB.pw_batch_davidson_init(self.handle, ptrs, lds))

    def step(self, precond: int = PW_PRECOND_TPA, net=None) -> int:
        nc = C.c_int32(0)
        _check(LIB.pw_batch_davidson_step(self.handle, int(precond), net.handle if net is not None else None,
                                          C.byref(nc)))
        return nc.value

    def run(self, psi0s, max_iter: int = 200, precond: int = PW_PRECOND_TPA, net=None) -> np.ndarray:
        """init + run of every solve; psi0s None continues every solve from its state."""
        ptrs, lds = self._blocks(psi0s) if psi0s is not None else (None, None)
        conv = np.zeros(len(self.solvers), dtype=np.int32)
        _check(LIB.pw_batch_davidson_run(self.handle, ptrs, lds, int(max_iter), int(precond),
                                         net.handle if net is not None else None,
                                         conv.ctypes.data_as(C.POINTER(C.c_int32))))
        return conv.astype(bool)

    def close(self):
        if self._h:
            LIB.pw_batch_davidson_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_davidson_solve(probs, psi0s, tol: float = 5e-9, nstreams: int = 4, max_subspace: int = 0,
                         max_iter: int = 200, precond: int = PW_PRECOND_TPA, net=None, refine=None,
                         refine_tol: float = None) -> list:
    """Davidson on every problem side by side over nstreams streams; per
    problem dict(theta, rho, iterations, n_hpsi, converged).  With
    ``refine`` (one problem per solve on the same sphere, e.g. the FP64
    forms): run to ``tol``, switch every solve to its refine problem and
    continue side by side to ``refine_tol``."""
    import torch
    solvers = [Davidson(p, int(x.shape[0]), max_subspace, tol) for p, x in zip(probs, psi0s)]
    streams = [torch.cuda.Stream() for _ in range(max(1, int(nstreams)))]
    torch.cuda.synchronize()
    b = BatchDavidson(solvers, streams)
    try:
        conv = b.run(psi0s, max_iter, precond, net)
        if refine is not None:
            first = [pw_davidson_query(d)["iterations"] for d in solvers]
            for d, p in zip(solvers, refine):
                pw_davidson_set_problem(d, p)
                pw_davidson_set_tol(d, refine_tol if refine_tol else tol)
            torch.cuda.synchronize()
            conv = b.run(None, max_iter, precond, net)
        out = []
        for i, (d, c) in enumerate(zip(solvers, conv)):
            r = pw_davidson_query(d)
            r["converged"] = bool(c)
            if refine is not None:
                r["iterations_first"] = first[i]
            out.append(r)
    finally:
        b.close()
        for d in solvers:
            d.close()
    return out


def pw_problem_autotune(prob: Problem, nbands: int, reps: int = 3, stream=None) -> float:
    ld = (prob.npw + 63) // 64 * 64
    nbytes = 2 * int(nbands) * ld * 16
    scratch = _workspace(nbytes)
    ms = C.c_double(0.0)
    _check(LIB.pw_problem_autotune(prob.handle, int(nbands), int(reps), C.c_void_p(scratch.data_ptr()),
                                   nbytes, _stream(stream), C.byref(ms)))
    del scratch
    return ms.value


def pw_problem_set_tuning(prob: Problem, plane_group: int, band_chunk: int, ksplit: int,
                          plane_kernel: int) -> None:
    _check(LIB.pw_problem_set_tuning(prob.handle, int(plane_group), int(band_chunk), int(ksplit),
                                     int(plane_kernel)))


def pw_problem_tuning(prob: Problem) -> dict:
    g, c, k, pk = C.c_int32(), C.c_int64(), C.c_int32(), C.c_int32()
    _check(LIB.pw_problem_tuning(prob.handle, C.byref(g), C.byref(c), C.byref(k), C.byref(pk)))
    return dict(plane_group=g.value, band_chunk=c.value, ksplit=k.value, plane_kernel=pk.value)


def pw_eigh(A, stream=None):
    """Eigen-decomposition of a Hermitian complex128 matrix (torch, column-major
    as stored: A[:, j] is column j) -> (w ascending, Z) on the GPU."""
    import torch
    m = int(A.shape[0])
    if A.dim() != 2 or A.shape[1] != m or A.dtype != torch.complex128 or not A.is_cuda:
        raise ValueError("A must be a square complex128 GPU tensor")
    At = A.t().contiguous()          # column-major storage of A
    nbytes = C.c_size_t(0)
    _check(LIB.pw_eigh_workspace(m, C.byref(nbytes)))
    work = torch.empty(int(nbytes.value), dtype=torch.uint8, device=A.device)
    w = torch.empty(m, dtype=torch.float64, device=A.device)
    Zt = torch.empty((m, m), dtype=torch.complex128, device=A.device)
    _check(LIB.pw_eigh(C.c_void_p(At.data_ptr()), m, m, C.c_void_p(w.data_ptr()),
                       C.c_void_p(Zt.data_ptr()), m, C.c_void_p(work.data_ptr()), nbytes.value,
                       _stream(stream)))
    return w, Zt.t()


class Lanczos:
    """Owner of a pw_lanczos chain set (Lanczos recursion on H, many chains in
    lockstep) and of its workspace."""

    def __init__(self, prob: Problem, nchains: int, max_steps: int):
        nbytes = C.c_size_t(0)
        _check(LIB.pw_lanczos_workspace_size(prob.handle, int(nchains), int(max_steps), C.byref(nbytes)))
        self.workspace = _workspace(nbytes.value)
        h = C.c_void_p()
        _check(LIB.pw_lanczos_create(prob.handle, int(nchains), int(max_steps),
                                     C.c_void_p(self.workspace.data_ptr()), nbytes.value, C.byref(h)))
        self._h = h
        self.prob = prob
        self.nchains = int(nchains)
        self.max_steps = int(max_steps)

    @property
    def handle(self):
        if not self._h:
            raise PwError(-1, "Lanczos chain set already destroyed")
        return self._h

    def start(self, v, stream=None) -> None:
        vp_, ld, nb = _band_block(v, "v", self.prob.npw)
        if nb < self.nchains:
            raise ValueError("v has fewer rows than chains")
        _check(LIB.pw_lanczos_start(self.handle, vp_, ld, _stream(stream)))

    def run(self, nsteps: int, stream=None) -> None:
        _check(LIB.pw_lanczos_run(self.handle, int(nsteps), _stream(stream)))

    def coefficients(self, stream=None):
        """(alpha [nchains][max_steps], beta [nchains][max_steps+1], steps done) as device tensors."""
        import torch
        a = torch.zeros((self.nchains, self.max_steps), dtype=torch.float64, device="cuda")
        b = torch.zeros((self.nchains, self.max_steps + 1), dtype=torch.float64, device="cuda")
        n = C.c_int32(0)
        _check(LIB.pw_lanczos_coefficients(self.handle, C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                                           C.byref(n), _stream(stream)))
        return a, b, n.value

    def resolvent(self, z, stream=None):
        """g [nchains][nz] (device complex128) at the points z (device complex128 [nz])."""
        import torch
        zc = z.contiguous()
        _dev_ptr(zc, torch.complex128, "z")
        g = torch.zeros((self.nchains, zc.numel()), dtype=torch.complex128, device="cuda")
        _check(LIB.pw_lanczos_resolvent(self.handle, C.c_void_p(zc.data_ptr()), int(zc.numel()),
                                        C.c_void_p(g.data_ptr()), _stream(stream)))
        return g

    def close(self):
        if self._h:
            LIB.pw_lanczos_destroy(self._h)
            self._h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- SCF loop
def _grid_array(t, prob: Problem, name):
    import torch
    ptr = _dev_ptr(t, torch.float64, name)
    if not t.is_contiguous() or tuple(t.shape) != tuple(prob.nr):
        raise ValueError(f"{name}: expected a contiguous float64 grid of shape {tuple(prob.nr)}")
    return ptr


def pw_density(prob: Problem, psi, f, n, stream=None) -> None:
    """n += Omega^-1 sum_b f[b] |u_b(r)|^2 (n: float64 grid [N0][N1][N2] on the GPU)."""
    ps, ld, nb = _band_block(psi, "psi", prob.npw)
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.shape != (nb,):
        raise ValueError("one weight per band")
    nbytes = C.c_size_t(0)
    _check(LIB.pw_density_workspace_size(prob.handle, C.byref(nbytes)))
    work = _workspace(nbytes.value)
    _check(LIB.pw_density(prob.handle, ps, ld, nb, f.ctypes.data_as(C.POINTER(C.c_double)),
                          _grid_array(n, prob, "n"), C.c_void_p(work.data_ptr()), nbytes.value, _stream(stream)))


def pw_hxc(prob: Problem, n, vion=None, stream=None):
    """(v, energies): v = vion + V_H[n] + V_x[n] on the grid, energies =
    (E_H, E_x, int v_x n)."""
    import torch
    nbytes = C.c_size_t(0)
    _check(LIB.pw_hxc_workspace_size(prob.handle, C.byref(nbytes)))
    work = _workspace(nbytes.value)
    v = torch.empty_like(n)
    e = np.zeros(3)
    _check(LIB.pw_hxc(prob.handle, _grid_array(n, prob, "n"),
                      _grid_array(vion, prob, "vion") if vion is not None else None,
                      _grid_array(v, prob, "v"), e.ctypes.data_as(C.POINTER(C.c_double)),
                      C.c_void_p(work.data_ptr()), nbytes.value, _stream(stream)))
    return v, e


def pw_problem_set_vloc(prob: Problem, v, stream=None) -> None:
    _check(LIB.pw_problem_set_vloc(prob.handle, _grid_array(v, prob, "v"), _stream(stream)))


class _ScfDesc(C.Structure):
    _fields_ = [("nk", C.c_int32), ("probs", C.POINTER(C.c_void_p)), ("davs", C.POINTER(C.c_void_p)),
                ("batch", C.c_void_p), ("kweights", C.POINTER(C.c_double)), ("vion", C.c_void_p),
                ("nel", C.c_double), ("sigma", C.c_double), ("alpha", C.c_double), ("kerker_q0", C.c_double),
                ("exx_alpha", C.c_double), ("exx_tol", C.c_double), ("exx_direct", C.c_int32)]


SCF_OUT = ("drho", "mu", "e_band", "e_hartree", "e_x", "vxc_n", "e_total", "free_energy", "e_xx", "outer")


class Scf:
    """Owner of a pw_scf and its workspace; keeps the problems, Davidson
    states, optional batch and V_ion alive with it."""

    def __init__(self, probs, davs, kweights, vion, nel: float, sigma: float, alpha: float, batch=None,
                 kerker_q0: float = 0.0, exx_alpha: float = 0.0, exx_tol: float = 1e-8, exx_direct: bool = False,
                 stream=None):
        n = len(probs)
        self._keep = (list(probs), list(davs), batch, vion)
        self._pp = (C.c_void_p * n)(*[p.handle.value for p in probs])
        self._dd = (C.c_void_p * n)(*[d.handle.value for d in davs])
        self._kw = np.ascontiguousarray(kweights, dtype=np.float64)
        d = _ScfDesc(n, self._pp, self._dd, batch.handle if batch is not None else None,
                     self._kw.ctypes.data_as(C.POINTER(C.c_double)), _grid_array(vion, probs[0], "vion"),
                     float(nel), float(sigma), float(alpha), float(kerker_q0), float(exx_alpha),
                     float(exx_tol), 1 if exx_direct else 0)
        nbytes = C.c_size_t(0)
        _check(LIB.pw_scf_workspace_size(C.byref(d), C.byref(nbytes)))
        self.workspace = _workspace(nbytes.value)
        h = C.c_void_p()
        _check(LIB.pw_scf_create(C.byref(d), C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                 _stream(stream), C.byref(h)))
        self._h = h
        self.prob0 = probs[0]

    @property
    def handle(self):
        if not self._h:
            raise PwError(-1, "SCF handle already destroyed")
        return self._h

    def step(self, dav_tol: float, dav_max_iter: int, tol: float) -> dict:
        out = np.zeros(10)
        c = C.c_int32(0)
        _check(LIB.pw_scf_step(self.handle, float(dav_tol), int(dav_max_iter), float(tol),
                               out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(c)))
        r = dict(zip(SCF_OUT, out.tolist()))
        r["converged"] = bool(c.value)
        return r

    def density(self, stream=None):
        import torch
        shape = tuple(self.prob0.nr)
        n_in = torch.empty(shape, dtype=torch.float64, device="cuda")
        n_out = torch.empty_like(n_in)
        _check(LIB.pw_scf_density(self.handle, C.c_void_p(n_in.data_ptr()), C.c_void_p(n_out.data_ptr()),
                                  _stream(stream)))
        return n_in, n_out

    def potential(self, stream=None):
        import torch
        v = torch.empty(tuple(self.prob0.nr), dtype=torch.float64, device="cuda")
        _check(LIB.pw_scf_potential(self.handle, C.c_void_p(v.data_ptr()), _stream(stream)))
        return v

    def close(self):
        if self._h:
            LIB.pw_scf_destroy(self._h)
            self._h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- exact exchange
def pw_vx(prob: Problem, psi_occ, w, phi, out, stream=None) -> None:
    """out = V_x phi (Gamma point) from the occupied bands psi_occ with weights w."""
    po, ldo, no = _band_block(psi_occ, "psi_occ", prob.npw)
    pp, ldp, nph = _band_block(phi, "phi", prob.npw)
    pq, ldq, nq = _band_block(out, "out", prob.npw)
    if nq < nph:
        raise ValueError("out has fewer bands than phi")
    w = np.ascontiguousarray(w, dtype=np.float64)
    if w.shape != (no,):
        raise ValueError("one weight per occupied band")
    nbytes = C.c_size_t(0)
    _check(LIB.pw_vx_workspace_size(prob.handle, no, C.byref(nbytes)))
    work = _workspace(nbytes.value)
    _check(LIB.pw_vx(prob.handle, po, ldo, no, w.ctypes.data_as(C.POINTER(C.c_double)), pp, ldp, nph, pq, ldq,
                     C.c_void_p(work.data_ptr()), nbytes.value, _stream(stream)))


def pw_ace_set(prob: Problem, psi_occ, w, alpha: float = 1.0, stream=None) -> None:
    """Attach alpha V_ace built from psi_occ to H psi; the zeta and projection
    buffers are allocated here and kept on the Problem object."""
    import torch
    po, ldo, no = _band_block(psi_occ, "psi_occ", prob.npw)
    w = np.ascontiguousarray(w, dtype=np.float64)
    if w.shape != (no,):
        raise ValueError("one weight per occupied band")
    ld = (prob.npw + 63) // 64 * 64
    zeta = torch.zeros((no, ld), dtype=torch.complex128, device="cuda")
    proj = torch.zeros((prob.max_bands, no), dtype=torch.complex128, device="cuda")
    nbytes = C.c_size_t(0)
    _check(LIB.pw_ace_workspace_size(prob.handle, no, C.byref(nbytes)))
    work = _workspace(nbytes.value)
    _check(LIB.pw_ace_set(prob.handle, po, ldo, no, w.ctypes.data_as(C.POINTER(C.c_double)), float(alpha),
                          C.c_void_p(zeta.data_ptr()), ld, C.c_void_p(proj.data_ptr()),
                          C.c_void_p(work.data_ptr()), nbytes.value, _stream(stream)))
    prob.ace = (zeta, proj)


def pw_vx_attach(prob: Problem, psi_occ, w, alpha: float = 1.0, stream=None) -> None:
    """Attach alpha V_x, applied directly, built on psi_occ (kept bound, with a
    scratch buffer, on the Problem object)."""
    po, ldo, no = _band_block(psi_occ, "psi_occ", prob.npw)
    w = np.ascontiguousarray(w, dtype=np.float64)
    if w.shape != (no,):
        raise ValueError("one weight per occupied band")
    nbytes = C.c_size_t(0)
    _check(LIB.pw_vx_workspace_size(prob.handle, no, C.byref(nbytes)))
    work = _workspace(nbytes.value)
    _check(LIB.pw_vx_attach(prob.handle, po, ldo, no, w.ctypes.data_as(C.POINTER(C.c_double)), float(alpha),
                            C.c_void_p(work.data_ptr()), nbytes.value, _stream(stream)))
    prob.ace = (psi_occ, work)


def pw_ace_clear(prob: Problem) -> None:
    _check(LIB.pw_ace_clear(prob.handle))
    prob.ace = None
