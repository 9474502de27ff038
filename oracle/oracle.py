"""ctypes shim over liboracle.so (test infrastructure only).

Every function takes a ``meshgen.Mesh`` in user numbering and numpy float64 arrays, and returns
numpy arrays.  Nothing here computes any part of the method: the arithmetic is in oracle.cpp.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


TABLE_U, TABLE_P, TABLE_ALL_FIXED, TABLE_ALL_ZEROGRAD = 0, 1, 2, 3
SCHEME_ONE, SCHEME_UPWIND, SCHEME_LINEAR = 0, 1, 2
OK, WARN_NOT_CONVERGED, WARN_BREAKDOWN = 0, 1, 2

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)


class OmMesh(C.Structure):
    _fields_ = [("nc", C.c_int32), ("nfi", C.c_int32), ("nfb", C.c_int32), ("npatch", C.c_int32),
                ("owner", _i32p), ("nbr", _i32p), ("Sf", _f64p), ("Cf", _f64p), ("C", _f64p),
                ("V", _f64p), ("w", _f64p), ("pstart", _i32p), ("psize", _i32p), ("putype", _i32p),
                ("pptype", _i32p), ("pwk", _i32p), ("nonorth", C.c_int32)]


# Non-orthogonal correction schemes (Sec. "Diffusive flux discretization"); a mesh selects one through
# mesh.meta["nonorth"] (default: over-relaxed).
NONORTH = {"overrelaxed": 0, "minimum": 1, "orthogonal": 2, "none": 3}


class OmPisoParams(C.Structure):
    _fields_ = [("nu", C.c_double), ("dt", C.c_double), ("n_corr", C.c_int32), ("tol_p", C.c_double),
                ("tol_u", C.c_double), ("maxit_p", C.c_int32), ("maxit_u", C.c_int32),
                ("p_ref_cell", C.c_int32), ("p_ref_value", C.c_double), ("tol_tangent", C.c_double),
                ("conv", C.c_int32), ("time", C.c_int32)]


# convection schemes (upwind implicit; the others by deferred correction, eq. deferred_correction)
CONV = {"upwind": 0, "linear": 1, "sou": 2, "quick": 3}
# time schemes (theta-method on the matrix part: 1, 0, 1/2)
TIME = {"backward_euler": 0, "forward_euler": 1, "crank_nicolson": 2}


_LIBS = {}
_VARIANT = "serial"


def use_threads(on=True):
    """Switch every later call to the all-threads timing build (liboracle_omp.so, OpenMP threads from
    OMP_NUM_THREADS) or back to the serial build the parity tests use."""
    global _VARIANT
    _VARIANT = "omp" if on else "serial"


def threads():
    """Host threads of the current build's Krylov kernels."""
    L = lib()
    L.oracle_threads.restype = C.c_int
    return L.oracle_threads()


def lib():
    if _VARIANT not in _LIBS:
        path = os.path.join(HERE, "liboracle_omp.so" if _VARIANT == "omp" else "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        L.oracle_version.restype = C.c_int
        if L.oracle_version() != 6:
            raise RuntimeError(f"{path} is stale (version {L.oracle_version()}); rebuild the oracle")
        _LIBS[_VARIANT] = L
    return _LIBS[_VARIANT]


def _p(a, t=_f64p):
    return None if a is None else a.ctypes.data_as(t)


class _Hold:
    """keeps numpy buffers referenced by an OmMesh alive"""


def om(mesh):
    """Build (and cache on the mesh object) the C view of a meshgen.Mesh, with the correction scheme
    named by mesh.meta["nonorth"]."""
    scheme = NONORTH[mesh.meta.get("nonorth", "overrelaxed")]
    cached = getattr(mesh, "_om", None)
    if cached is not None and cached[3] == scheme:
        return cached[0]
    h = _Hold()
    h.owner = np.ascontiguousarray(mesh.owner, dtype=np.int32)
    h.nbr = np.ascontiguousarray(mesh.neighbour, dtype=np.int32)
    h.Sf = np.ascontiguousarray(mesh.Sf, dtype=np.float64)
    h.Cf = np.ascontiguousarray(mesh.Cf, dtype=np.float64)
    h.C = np.ascontiguousarray(mesh.C, dtype=np.float64)
    h.V = np.ascontiguousarray(mesh.V, dtype=np.float64)
    h.w = np.ascontiguousarray(mesh.w, dtype=np.float64)
    h.pstart = np.array([p.start for p in mesh.patches], dtype=np.int32)
    h.psize = np.array([p.size for p in mesh.patches], dtype=np.int32)
    h.putype = np.array([p.u_type for p in mesh.patches], dtype=np.int32)
    h.pptype = np.array([p.p_type for p in mesh.patches], dtype=np.int32)
    h.pwk = np.array([p.wk_id for p in mesh.patches], dtype=np.int32)
    s = OmMesh(mesh.n_cells, mesh.n_internal_faces, mesh.n_boundary_faces, len(mesh.patches),
               _p(h.owner, _i32p), _p(h.nbr, _i32p), _p(h.Sf), _p(h.Cf), _p(h.C), _p(h.V), _p(h.w),
               _p(h.pstart, _i32p), _p(h.psize, _i32p), _p(h.putype, _i32p), _p(h.pptype, _i32p),
               _p(h.pwk, _i32p), scheme)
    mesh._om = (C.byref(s), s, h, scheme)
    return mesh._om[0]


def _f(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def renumber(mesh, rcm=True):
    L = lib()
    nc, nfi, nfb = mesh.n_cells, mesh.n_internal_faces, mesh.n_boundary_faces
    out = dict(cell_perm=np.empty(nc, np.int32), face_perm=np.empty(nfi, np.int32),
               face_flip=np.empty(nfi, np.uint8), owner=np.empty(nfi, np.int32), neighbour=np.empty(nfi, np.int32),
               own_start=np.empty(nc + 1, np.int32), losort=np.empty(nfi, np.int32),
               losort_start=np.empty(nc + 1, np.int32), bface_perm=np.empty(nfb, np.int32),
               bowner=np.empty(nfb, np.int32))
    rc = L.oracle_renumber(om(mesh), int(rcm), *[_p(out[k], C.c_void_p) for k in
                           ("cell_perm", "face_perm", "face_flip", "owner", "neighbour", "own_start", "losort",
                            "losort_start", "bface_perm", "bowner")])
    assert rc == 0
    return out


def bandwidth(mesh):
    return int(lib().oracle_bandwidth(om(mesh)))


def geometry(mesh):
    nfi, nfb = mesh.n_internal_faces, mesh.n_boundary_faces
    delta, k, db = np.empty(nfi), np.empty((nfi, 3)), np.empty(nfb)
    lib().oracle_geometry(om(mesh), _p(delta), _p(k), _p(db))
    return delta, k, db


def interp(mesh, phi, phib=None, table=TABLE_ALL_FIXED):
    phi = _f(phi)
    ncomp = 1 if phi.ndim == 1 else phi.shape[1]
    out = np.empty((mesh.n_faces, ncomp)) if ncomp > 1 else np.empty(mesh.n_faces)
    lib().oracle_interp(om(mesh), ncomp, table, _p(phi), _p(_f(phib)), _p(out))
    return out


def grad(mesh, phi, phib=None, table=TABLE_ALL_FIXED):
    phi = _f(phi)
    ncomp = 1 if phi.ndim == 1 else phi.shape[1]
    out = np.empty((mesh.n_cells, 3)) if ncomp == 1 else np.empty((mesh.n_cells, ncomp, 3))
    lib().oracle_grad(om(mesh), ncomp, table, _p(phi), _p(_f(phib)), _p(out))
    return out


def grad_surface(mesh, phif, table=TABLE_ALL_FIXED):
    phif = _f(phif)
    ncomp = 1 if phif.ndim == 1 else phif.shape[1]
    out = np.empty((mesh.n_cells, 3)) if ncomp == 1 else np.empty((mesh.n_cells, ncomp, 3))
    lib().oracle_grad_surface(om(mesh), ncomp, table, _p(phif), _p(out))
    return out


def div(mesh, flux, psi=None, psib=None, scheme=SCHEME_ONE, table=TABLE_ALL_FIXED, absterms=False):
    flux = _f(flux)
    if psi is None:
        psi = np.zeros(mesh.n_cells)
    psi = _f(psi)
    ncomp = 1 if psi.ndim == 1 else psi.shape[1]
    out = np.empty((mesh.n_cells, ncomp)) if ncomp > 1 else np.empty(mesh.n_cells)
    fn = lib().oracle_div_absterms if absterms else lib().oracle_div
    fn(om(mesh), scheme, ncomp, table, _p(flux), _p(psi), _p(_f(psib)), _p(out))
    return out


def laplacian(mesh, phi, g, phib=None, gamma=None, table=TABLE_ALL_FIXED):
    out = np.empty(mesh.n_cells)
    lib().oracle_laplacian(om(mesh), table, _p(_f(gamma)), _p(_f(phi)), _p(_f(g)), _p(_f(phib)), _p(out))
    return out


def spmv(mesh, diag, upper, lower, x, transpose=False):
    x = _f(x)
    ncomp = 1 if x.ndim == 1 else x.shape[1]
    y = np.empty_like(x)
    lib().oracle_spmv(om(mesh), ncomp, int(transpose), _p(_f(diag)), _p(_f(upper)), _p(_f(lower)), _p(x), _p(y))
    return y


def assemble_laplace(mesh, phib=None, gamma=None, table=TABLE_ALL_FIXED):
    nc, nfi = mesh.n_cells, mesh.n_internal_faces
    diag, upper, rhs = np.empty(nc), np.empty(nfi), np.empty(nc)
    if phib is None:
        phib = np.zeros(mesh.n_boundary_faces)
    lib().oracle_assemble_laplace(om(mesh), table, _p(_f(gamma)), _p(_f(phib)), _p(diag), _p(upper), _p(rhs))
    return diag, upper, rhs


def assemble_momentum(mesh, nu, dt, phi, U, Ub):
    nc, nfi = mesh.n_cells, mesh.n_internal_faces
    diag, upper, lower, b = np.empty(nc), np.empty(nfi), np.empty(nfi), np.empty((nc, 3))
    lib().oracle_assemble_momentum(om(mesh), C.c_double(nu), C.c_double(dt), _p(_f(phi)), _p(_f(U)), _p(_f(Ub)),
                                   _p(diag), _p(upper), _p(lower), _p(b))
    return diag, upper, lower, b


def pcg(mesh, diag, upper, b, x0=None, tol=1e-8, maxit=2000):
    x = np.zeros(mesh.n_cells) if x0 is None else _f(x0).copy()
    it, res = C.c_int32(0), C.c_double(0)
    st = lib().oracle_pcg(om(mesh), _p(_f(diag)), _p(_f(upper)), _p(_f(b)), _p(x), C.c_double(tol), int(maxit),
                          C.byref(it), C.byref(res))
    return x, it.value, res.value, st


def bicgstab(mesh, diag, upper, lower, b, x0=None, tol=1e-8, maxit=500):
    b = _f(b)
    ncomp = 1 if b.ndim == 1 else b.shape[1]
    x = np.zeros_like(b) if x0 is None else _f(x0).copy()
    it, res = np.zeros(ncomp, np.int32), np.zeros(ncomp)
    st = lib().oracle_bicgstab(om(mesh), ncomp, _p(_f(diag)), _p(_f(upper)), _p(_f(lower)), _p(b), _p(x),
                               C.c_double(tol), int(maxit), _p(it, _i32p), _p(res))
    return x, it, res, st


def transport_scalar(mesh, phi, c, cb, D, dt, table=TABLE_U, tol=1e-8, maxit=500, conv="upwind",
                     time="backward_euler"):
    """One step of a passive scalar with face flux phi; returns (c_new, iters, res, status)."""
    x = np.array(c, dtype=np.float64, copy=True)
    it, rs = C.c_int32(0), C.c_double(0.0)
    st = lib().oracle_transport_scalar(om(mesh), int(table), CONV[conv], TIME[time], C.c_double(D), C.c_double(dt),
                                       _p(_f(phi)), _p(_f(cb)), _p(x), C.c_double(tol), int(maxit), C.byref(it),
                                       C.byref(rs))
    return x, it.value, rs.value, st


def deferred_correction(mesh, conv, flux, phi, g):
    """Explicit deferred-correction source -sum sigma F (phi^HO - phi^U) of scheme conv; phi [nc] or
    [nc, ncomp], g the cell gradients [nc, 3] or [nc, ncomp, 3]."""
    phi = _f(phi)
    ncomp = 1 if phi.ndim == 1 else phi.shape[1]
    out = np.empty_like(phi)
    lib().oracle_deferred_correction(om(mesh), CONV[conv], ncomp, _p(_f(flux)), _p(phi), _p(_f(g)), _p(out))
    return out


def initial_flux(mesh, U, Ub):
    phi = np.empty(mesh.n_faces)
    lib().oracle_initial_flux(om(mesh), _p(_f(U)), _p(_f(Ub)), _p(phi))
    return phi


def piso_params(nu, dt, n_corr=2, tol_p=1e-8, tol_u=1e-8, maxit_p=2000, maxit_u=500, p_ref_cell=0, p_ref_value=0.0,
                tol_tangent=1e-13, conv="upwind", time="backward_euler"):
    return OmPisoParams(nu, dt, n_corr, tol_p, tol_u, maxit_p, maxit_u, p_ref_cell, p_ref_value, tol_tangent,
                        CONV[conv], TIME[time])


def piso_run(mesh, prm, U, p, phi, Ub, pb, wk=None, pc=None, nsteps=1, trace=False):
    """Returns (U, p, phi, pc, iters[nsteps, 3+n_corr], res[nsteps, 3+n_corr], status); with trace=True
    also (Ustar[nsteps, nc, 3], pcorr[nsteps, n_corr, nc]): the solution of every linear solve."""
    U, p, phi = _f(U).copy(), _f(p).copy(), _f(phi).copy()
    wk = np.zeros((0, 3)) if wk is None else _f(wk)
    nwk = wk.shape[0]
    pc = np.zeros(max(nwk, 1)) if pc is None else _f(pc).copy()
    per = 3 + prm.n_corr
    iters = np.zeros((nsteps, per), np.int32)
    res = np.zeros((nsteps, per))
    Us = np.zeros((nsteps, mesh.n_cells, 3)) if trace else None
    pcs = np.zeros((nsteps, prm.n_corr, mesh.n_cells)) if trace else None
    st = lib().oracle_piso_run_trace(om(mesh), C.byref(prm), _p(_f(Ub)), _p(_f(pb)),
                                     _p(np.ascontiguousarray(wk.ravel())), nwk, _p(pc), _p(U), _p(p), _p(phi),
                                     int(nsteps), _p(iters, _i32p), _p(res), _p(Us), _p(pcs))
    if trace:
        return U, p, phi, pc[:nwk], iters, res, st, Us, pcs
    return U, p, phi, pc[:nwk], iters, res, st


def piso_check_step(mesh, prm, U, p, phi, Ub, pb, Ustar, pcorr, wk=None, pc=None):
    """One step from (U, p, phi, pc) in verification mode: the predictor solution Ustar[nc, 3] and the
    pressure after each corrector pcorr[n_corr, nc] are supplied instead of solved.  Returns
    (U, p, phi, pc, res_u[3], res_p[n_corr]): the state the step computes from those solutions and the
    true relative residual ||b - A x||_2 / ||b||_2 of each of its linear systems."""
    U, p, phi = _f(U).copy(), _f(p).copy(), _f(phi).copy()
    wk = np.zeros((0, 3)) if wk is None else _f(wk)
    nwk = wk.shape[0]
    pc = np.zeros(max(nwk, 1)) if pc is None else _f(pc).copy()
    Ustar = _f(Ustar)
    pcorr = _f(pcorr)
    assert Ustar.size == 3 * mesh.n_cells and pcorr.size == prm.n_corr * mesh.n_cells
    res_u, res_p = np.zeros(3), np.zeros(prm.n_corr)
    st = lib().oracle_piso_check_step(om(mesh), C.byref(prm), _p(_f(Ub)), _p(_f(pb)),
                                      _p(np.ascontiguousarray(wk.ravel())), nwk, _p(pc), _p(U), _p(p), _p(phi),
                                      _p(Ustar), _p(pcorr), _p(res_u), _p(res_p))
    if st != 0:
        raise ValueError("oracle_piso_check_step: n_corr out of range")
    return U, p, phi, pc[:nwk], res_u, res_p


def piso_tangent(mesh, prm, U, p, phi, Ub, pb, wk, pc, nsteps, dwk=None, dU0=None, dp0=None, dphi0=None, dpc0=None,
                 nd=None, dUb=None):
    """Forward-mode tangents of the final state.  Seeds have a leading direction axis (nd <= 10); dUb
    seeds the fixed velocity boundary values [nd, Fb, 3]."""
    U, p, phi = _f(U).copy(), _f(p).copy(), _f(phi).copy()
    wk = _f(wk).reshape(-1, 3)
    nwk = wk.shape[0]
    pc = _f(pc).copy() if nwk else np.zeros(1)
    seeds = [s for s in (dwk, dU0, dp0, dphi0, dpc0, dUb) if s is not None]
    if nd is None:
        nd = seeds[0].shape[0] if seeds else 0
    nc, nf = mesh.n_cells, mesh.n_faces
    tU, tp, tphi, tpc = np.zeros((nd, nc, 3)), np.zeros((nd, nc)), np.zeros((nd, nf)), np.zeros((nd, max(nwk, 1)))

    def sd(a):
        return None if a is None else _p(np.ascontiguousarray(np.asarray(a, np.float64)))
    hold = [None if a is None else np.ascontiguousarray(np.asarray(a, np.float64))
            for a in (dwk, dU0, dp0, dphi0, dpc0, dUb)]
    st = lib().oracle_piso_tangent(om(mesh), C.byref(prm), _p(_f(Ub)), _p(_f(pb)),
                                   _p(np.ascontiguousarray(wk.ravel())), nwk, _p(pc), _p(U), _p(p), _p(phi),
                                   int(nsteps), int(nd), *[None if a is None else _p(a) for a in hold],
                                   _p(tU), _p(tp), _p(tphi), _p(tpc))
    return dict(U=U, p=p, phi=phi, pc=pc[:nwk], tU=tU, tp=tp, tphi=tphi, tpc=tpc[:, :nwk], status=st)
