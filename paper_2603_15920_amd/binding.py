"""ctypes binding of libdifvm.so (include/difvm.h).  Argument marshalling only: every computation runs
in the library's HIP kernels.  Device arrays are contiguous torch tensors on the context's device;
torch supplies memory and the stream.

The ``difvm_*`` functions mirror the C entry points one to one (raising ``DifvmError`` on a negative
status and returning warnings); ``Context``, ``Mesh`` and ``Piso`` own the C handles.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdifvm.so")

F64, F32 = 0, 1
BC_U, BC_P, BC_ALL_FIXED, BC_ALL_ZEROGRAD = 0, 1, 2, 3
SCHEME_ONE, SCHEME_UPWIND, SCHEME_LINEAR = 0, 1, 2
# convection schemes of the PISO predictor and scalar transport (deferred correction beyond upwind)
CONV = {"upwind": 0, "linear": 1, "sou": 2, "quick": 3}
# time schemes (theta-method on the predictor's matrix part: 1, 0, 1/2)
TIME = {"backward_euler": 0, "forward_euler": 1, "crank_nicolson": 2}
# pressure preconditioners
PRECOND = {"jacobi": 0, "amg": 1}
KIND_CELL, KIND_FACE, KIND_FACE_FLUX, KIND_BFACE = 0, 1, 2, 3
TO_INTERNAL, FROM_INTERNAL = 0, 1
RENUMBER_RCM = 1
# non-orthogonal correction schemes (a two-bit field of the mesh flags), keyed like mesh.meta["nonorth"]
NONORTH = {"overrelaxed": 0, "minimum": 2, "orthogonal": 4, "none": 6}
OK, WARN_NOT_CONVERGED, WARN_BREAKDOWN = 0, 1, 2
TUNE_KNOBS = ["interp_f64", "interp_f32", "grad_f64", "grad_f32", "div_f64", "div_f32", "laplacian_f64",
              "laplacian_f32", "ldu_spmv_f64", "ldu_spmv_f32", "pcg_grid"]
TUNE_PCG_GRID = 10
ERR_INVALID_ARG, ERR_INVALID_MESH, ERR_HIP, ERR_OOM, ERR_UNSUPPORTED, ERR_NONFINITE = -1, -2, -3, -4, -5, -6

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)
_vp = C.c_void_p


class DifvmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"difvm status {status}: {msg}")
        self.status = status


class Patch(C.Structure):
    _fields_ = [("start", C.c_int32), ("size", C.c_int32), ("u_type", C.c_int32), ("p_type", C.c_int32),
                ("windkessel_id", C.c_int32)]


class MeshDesc(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("n_cells", C.c_int32), ("n_internal_faces", C.c_int32),
                ("n_boundary_faces", C.c_int32), ("n_patches", C.c_int32), ("owner", _i32p), ("neighbour", _i32p),
                ("Sf", _f64p), ("Cf", _f64p), ("C", _f64p), ("V", _f64p), ("w", _f64p), ("patches", C.POINTER(Patch))]


class MeshInfo(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n_cells", "n_internal_faces", "n_boundary_faces", "n_patches", "n_slices",
                                          "n_slots", "bandwidth_in", "bandwidth_out", "n_windkessel", "has_fixed_p",
                                          "n_segments")]


class PartInfo(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n_parts", "cell_lo", "cell_hi", "n_owned", "n_ghost", "n_internal_faces",
                                          "n_boundary_faces", "n_send", "n_neighbours")]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int32), ("total_ms", C.c_double)]


class Ldu(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("diag", _vp), ("upper", _vp), ("lower", _vp)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32 * 3), ("residual", C.c_double * 3), ("status", C.c_int32)]


class PisoParams(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("nu", C.c_double), ("dt", C.c_double), ("n_corr", C.c_int32),
                ("tol_p", C.c_double), ("tol_u", C.c_double), ("maxit_p", C.c_int32), ("maxit_u", C.c_int32),
                ("p_ref_cell", C.c_int32), ("p_ref_value", C.c_double), ("conv", C.c_int32), ("time", C.c_int32),
                ("precond", C.c_int32)]


class StepStats(C.Structure):
    _fields_ = [("it_u", C.c_int32 * 3), ("res_u", C.c_double * 3), ("it_p", C.c_int32 * 8), ("res_p", C.c_double * 8),
                ("status", C.c_int32)]


_LIB = None

_SIGS = {
    "difvm_abi_version": (C.c_int, []),
    "difvm_last_error": (C.c_char_p, []),
    "difvm_ctx_create": (C.c_int32, [C.c_int, _vp, C.POINTER(_vp)]),
    "difvm_ctx_set_stream": (C.c_int32, [_vp, _vp]),
    "difvm_ctx_destroy": (C.c_int32, [_vp]),
    "difvm_ctx_set_allocator": (C.c_int32, [_vp, _vp, _vp, _vp]),
    "difvm_ctx_profile": (C.c_int32, [_vp, C.c_int]),
    "difvm_ctx_profile_phases": (C.c_int32, [_vp, C.c_int]),
    "difvm_ctx_profile_read": (C.c_int32, [_vp, C.POINTER(KernelTime), C.c_int32, C.POINTER(C.c_int32)]),
    "difvm_mesh_renumber_host": (C.c_int32, [C.POINTER(MeshDesc), C.c_uint32] + [_vp] * 14),
    "difvm_mesh_create": (C.c_int32, [_vp, C.POINTER(MeshDesc), C.c_uint32, C.POINTER(_vp)]),
    "difvm_mesh_create_segments": (C.c_int32, [_vp, C.POINTER(MeshDesc), C.c_uint32, C.c_int32, _i32p,
                                               C.POINTER(_vp)]),
    "difvm_mesh_get_info": (C.c_int32, [_vp, C.POINTER(MeshInfo)]),
    "difvm_partition_create": (C.c_int32, [C.POINTER(MeshDesc), C.c_uint32, C.c_int32, C.POINTER(_vp)]),
    "difvm_partition_destroy": (C.c_int32, [_vp]),
    "difvm_partition_info": (C.c_int32, [_vp, C.c_int32, C.POINTER(PartInfo)]),
    "difvm_partition_maps": (C.c_int32, [_vp, C.c_int32] + [_i32p] * 6),
    "difvm_mesh_create_part": (C.c_int32, [_vp, _vp, C.c_int32, C.POINTER(_vp)]),
    "difvm_halo_pack": (C.c_int32, [_vp, C.c_int, C.c_int, _vp, _vp]),
    "difvm_halo_unpack": (C.c_int32, [_vp, C.c_int, C.c_int, _vp, _vp]),
    "difvm_mesh_set_launch": (C.c_int32, [_vp, C.c_int32, C.c_int32]),
    "difvm_mesh_get_launch": (C.c_int32, [_vp, C.c_int32, C.POINTER(C.c_int32)]),
    "difvm_tune": (C.c_int32, [_vp, C.c_char_p, C.POINTER(C.c_int32)]),
    "difvm_mesh_destroy": (C.c_int32, [_vp]),
    "difvm_permute": (C.c_int32, [_vp, C.c_int, C.c_int, C.c_int, C.c_int, _vp, _vp]),
    "difvm_op_interp": (C.c_int32, [_vp, C.c_int, C.c_int, C.c_int, _vp, _vp, _vp]),
    "difvm_op_grad": (C.c_int32, [_vp, C.c_int, C.c_int, C.c_int, _vp, _vp, _vp]),
    "difvm_op_div": (C.c_int32, [_vp, C.c_int, C.c_int, C.c_int, C.c_int, _vp, _vp, _vp, _vp]),
    "difvm_op_deferred_correction": (C.c_int32, [_vp, C.c_int, C.c_int, C.c_int, _vp, _vp, _vp, _vp]),
    "difvm_op_laplacian": (C.c_int32, [_vp, C.c_int, C.c_int, _vp, _vp, _vp, _vp, _vp]),
    "difvm_ldu_spmv": (C.c_int32, [_vp, C.c_int, C.c_int, C.POINTER(Ldu), _vp, _vp]),
    "difvm_ldu_assemble_laplace": (C.c_int32, [_vp, C.c_int, _vp, _vp, C.POINTER(Ldu), _vp]),
    "difvm_ldu_assemble_momentum": (C.c_int32, [_vp, C.c_double, C.c_double, _vp, _vp, _vp, C.POINTER(Ldu), _vp]),
    "difvm_ldu_assemble_momentum_noalloc": (C.c_int32, [_vp, C.c_double, C.c_double, _vp, _vp, _vp, C.POINTER(Ldu),
                                                        _vp]),
    "difvm_solve_pcg": (C.c_int32, [_vp, C.POINTER(Ldu), _vp, _vp, C.c_double, C.c_int32, C.POINTER(SolveStats)]),
    "difvm_amg_create": (C.c_int32, [_vp, C.POINTER(Ldu), C.POINTER(_vp)]),
    "difvm_amg_destroy": (C.c_int32, [_vp]),
    "difvm_amg_setup_host": (C.c_int32, [C.c_int32, _i32p, _i32p, _f64p, _f64p, _i32p, _i32p, C.c_int32, _i32p]),
    "difvm_amg_levels": (C.c_int32, [_vp, _i32p, C.c_int32, _i32p]),
    "difvm_amg_apply": (C.c_int32, [_vp, _vp, _vp]),
    "difvm_solve_pcg_amg": (C.c_int32, [_vp, C.POINTER(Ldu), _vp, _vp, C.c_double, C.c_int32, C.POINTER(SolveStats)]),
    "difvm_piso_rebuild_preconditioner": (C.c_int32, [_vp]),
    "difvm_solve_bicgstab": (C.c_int32, [_vp, C.POINTER(Ldu), C.c_int, _vp, _vp, C.c_double, C.c_int32,
                                         C.POINTER(SolveStats)]),
    "difvm_piso_create": (C.c_int32, [_vp, C.POINTER(PisoParams), C.POINTER(_vp)]),
    "difvm_piso_destroy": (C.c_int32, [_vp]),
    "difvm_piso_set_boundary": (C.c_int32, [_vp, _vp, _vp]),
    "difvm_piso_set_windkessel": (C.c_int32, [_vp, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double]),
    "difvm_piso_set_viscosity": (C.c_int32, [_vp, C.c_int32, _f64p]),
    "difvm_piso_segment_stats": (C.c_int32, [_vp, C.c_int32, C.POINTER(StepStats)]),
    "difvm_piso_transport_scalar": (C.c_int32, [_vp, C.c_double, C.c_int32, _vp, _vp, C.POINTER(SolveStats)]),
    "difvm_piso_set_graph": (C.c_int32, [_vp, C.c_int32, C.c_int32]),
    "difvm_piso_graph_info": (C.c_int32, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "difvm_piso_set_state": (C.c_int32, [_vp, _vp, _vp, _vp]),
    "difvm_piso_get_state": (C.c_int32, [_vp, _vp, _vp, _vp, _f64p]),
    "difvm_piso_step": (C.c_int32, [_vp, C.c_int32, C.POINTER(StepStats)]),
    "difvm_piso_step_trace": (C.c_int32, [_vp, _vp, _vp, C.POINTER(StepStats)]),
    "difvm_piso_precond_info": (C.c_int32, [_vp, _i32p, _i32p, C.c_int32, _f64p]),
    "difvm_tape_create": (C.c_int32, [_vp, C.c_int32, C.c_int32, C.POINTER(_vp)]),
    "difvm_tape_destroy": (C.c_int32, [_vp]),
    "difvm_piso_forward_record": (C.c_int32, [_vp, _vp, C.POINTER(StepStats)]),
    "difvm_piso_adjoint": (C.c_int32, [_vp, _vp, _vp, _vp, _vp, _f64p, C.c_double, _vp, _vp, _vp, _f64p, _f64p]),
    "difvm_tape_boundary_cotangent": (C.c_int32, [_vp, _vp]),
    "difvm_tape_set_graph": (C.c_int32, [_vp, C.c_int32, C.c_int32]),
    "difvm_tape_graph_info": (C.c_int32, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
}


def lib():
    """Load libdifvm.so (built in place by paper_2603_15920_amd/build.py).  Fails loudly if absent."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python paper_2603_15920_amd/build.py`")
        # torch first: its bundled HIP runtime then serves this library too (same soname).  Loaded the
        # other way round, the process holds two HIP runtimes and the second finds no device.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _check(status, name):
    if status < 0:
        raise DifvmError(status, f"{name}: {lib().difvm_last_error().decode()}")
    return status


def _ptr(t):
    """data pointer of a contiguous torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("device arrays must be contiguous")
    return C.c_void_p(t.data_ptr())


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


# ------------------------------------------------------------------------------------------------
# one-to-one wrappers of the C entry points
# ------------------------------------------------------------------------------------------------
def difvm_abi_version():
    return lib().difvm_abi_version()


def difvm_ctx_create(device=0, hip_stream=None):
    out = _vp()
    _check(lib().difvm_ctx_create(int(device), hip_stream, C.byref(out)), "difvm_ctx_create")
    return out


def difvm_ctx_set_stream(ctx, hip_stream):
    _check(lib().difvm_ctx_set_stream(ctx, hip_stream), "difvm_ctx_set_stream")


# allocator callbacks of difvm_ctx_set_allocator: void* alloc(size_t, void* stream, void* user) and
# void free(void*, void* stream, void* user)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


def difvm_ctx_set_allocator(ctx, alloc_fn, free_fn):
    """alloc_fn / free_fn: ALLOC_FN / FREE_FN objects (the caller keeps them alive), or both None."""
    _check(lib().difvm_ctx_set_allocator(ctx, C.cast(alloc_fn, _vp) if alloc_fn else None,
                                         C.cast(free_fn, _vp) if free_fn else None, None),
           "difvm_ctx_set_allocator")


class TorchAllocator:
    """Routes the library's device memory through torch's caching allocator (the blocks show up in
    torch.cuda.memory_allocated and are reused by torch after the library returns them).  Counts the
    calls.  After interpreter shutdown has begun, frees are dropped (the process is ending)."""

    def __init__(self, device):
        import torch
        self.device = int(device)
        self.n_alloc = 0
        self.n_free = 0
        self.live = {}
        self._torch = torch

        def alloc(nbytes, stream, user):
            try:
                p = self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
            except Exception:  # an exception must not cross the C boundary: NULL means out of memory
                return None
            self.n_alloc += 1
            self.live[p] = int(nbytes)
            return p

        def free(ptr, stream, user):
            if _SHUTDOWN or not ptr:
                return
            try:
                self._torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:
                return
            self.n_free += 1
            self.live.pop(int(ptr), None)

        self.alloc_fn = ALLOC_FN(alloc)
        self.free_fn = FREE_FN(free)

    def counts(self):
        return self.n_alloc, self.n_free


_SHUTDOWN = False


def _mark_shutdown():
    global _SHUTDOWN
    _SHUTDOWN = True


import atexit  # noqa: E402

atexit.register(_mark_shutdown)


def difvm_ctx_destroy(ctx):
    _check(lib().difvm_ctx_destroy(ctx), "difvm_ctx_destroy")


def difvm_ctx_profile(ctx, every_nth):
    """every_nth >= 1: time every n-th launch of each PCG kernel with HIP events; 0: off."""
    _check(lib().difvm_ctx_profile(ctx, int(every_nth)), "difvm_ctx_profile")


def difvm_ctx_profile_phases(ctx, enable):
    """enable != 0: time the phases of every eager PISO step ("step: ..." names); 0: off."""
    _check(lib().difvm_ctx_profile_phases(ctx, int(enable)), "difvm_ctx_profile_phases")


def difvm_ctx_profile_read(ctx):
    """{kernel name: (launches, total ms)} since the last read (synchronises)."""
    buf = (KernelTime * 64)()
    n = C.c_int32(0)
    _check(lib().difvm_ctx_profile_read(ctx, buf, 64, C.byref(n)), "difvm_ctx_profile_read")
    return {buf[k].name.decode(): (buf[k].launches, buf[k].total_ms) for k in range(min(n.value, 64))}


class _DescHolder:
    pass


def mesh_desc(mesh):
    """difvm_mesh_desc over a meshgen.Mesh (host arrays kept alive by the returned holder)."""
    h = _DescHolder()
    h.owner = np.ascontiguousarray(mesh.owner, dtype=np.int32)
    h.nbr = np.ascontiguousarray(mesh.neighbour, dtype=np.int32)
    h.Sf = np.ascontiguousarray(mesh.Sf, dtype=np.float64)
    h.Cf = np.ascontiguousarray(mesh.Cf, dtype=np.float64)
    h.C = np.ascontiguousarray(mesh.C, dtype=np.float64)
    h.V = np.ascontiguousarray(mesh.V, dtype=np.float64)
    h.w = None if mesh.w is None else np.ascontiguousarray(mesh.w, dtype=np.float64)
    h.patches = (Patch * max(1, len(mesh.patches)))(*[Patch(p.start, p.size, p.u_type, p.p_type, p.wk_id)
                                                       for p in mesh.patches])
    h.desc = MeshDesc(C.sizeof(MeshDesc), mesh.n_cells, mesh.n_internal_faces, mesh.n_boundary_faces,
                      len(mesh.patches), h.owner.ctypes.data_as(_i32p), h.nbr.ctypes.data_as(_i32p),
                      h.Sf.ctypes.data_as(_f64p), h.Cf.ctypes.data_as(_f64p), h.C.ctypes.data_as(_f64p),
                      h.V.ctypes.data_as(_f64p), None if h.w is None else h.w.ctypes.data_as(_f64p), h.patches)
    return h


def difvm_mesh_renumber_host(mesh, flags=RENUMBER_RCM, geometry=False):
    """Host-only renumbering; returns a dict of numpy arrays (no device used)."""
    h = mesh_desc(mesh)
    nc, nfi, nfb = mesh.n_cells, mesh.n_internal_faces, mesh.n_boundary_faces
    out = dict(cell_perm=np.empty(nc, np.int32), face_perm=np.empty(nfi, np.int32), face_flip=np.empty(nfi, np.uint8),
               owner=np.empty(nfi, np.int32), neighbour=np.empty(nfi, np.int32), own_start=np.empty(nc + 1, np.int32),
               losort=np.empty(nfi, np.int32), losort_start=np.empty(nc + 1, np.int32),
               bface_perm=np.empty(nfb, np.int32), bowner=np.empty(nfb, np.int32))
    keys = list(out)
    if geometry:
        out.update(S=np.empty((nfi + nfb, 3)), w=np.empty(nfi), delta=np.empty(nfi + nfb), k=np.empty((nfi, 3)))
    ptrs = [out[k].ctypes.data_as(_vp) for k in keys]
    g = [out[k].ctypes.data_as(_vp) if geometry else None for k in ("S", "w", "delta", "k")]
    _check(lib().difvm_mesh_renumber_host(C.byref(h.desc), int(flags), *ptrs, *g), "difvm_mesh_renumber_host")
    return out


def difvm_mesh_create(ctx, mesh, flags=RENUMBER_RCM):
    h = mesh_desc(mesh)
    out = _vp()
    _check(lib().difvm_mesh_create(ctx, C.byref(h.desc), int(flags), C.byref(out)), "difvm_mesh_create")
    return out


def difvm_mesh_create_segments(ctx, mesh, seg_cell_start, flags=RENUMBER_RCM):
    h = mesh_desc(mesh)
    starts = np.ascontiguousarray(seg_cell_start, dtype=np.int32)
    out = _vp()
    _check(lib().difvm_mesh_create_segments(ctx, C.byref(h.desc), int(flags), int(starts.size - 1),
                                            starts.ctypes.data_as(_i32p), C.byref(out)), "difvm_mesh_create_segments")
    return out


def difvm_partition_create(mesh, n_parts, flags=RENUMBER_RCM):
    h = mesh_desc(mesh)
    out = _vp()
    _check(lib().difvm_partition_create(C.byref(h.desc), int(flags), int(n_parts), C.byref(out)),
           "difvm_partition_create")
    return out


def difvm_partition_destroy(part):
    _check(lib().difvm_partition_destroy(part), "difvm_partition_destroy")


def difvm_partition_info(part, p):
    info = PartInfo()
    _check(lib().difvm_partition_info(part, int(p), C.byref(info)), "difvm_partition_info")
    return {n: getattr(info, n) for n, _ in PartInfo._fields_}


def difvm_partition_maps(part, p):
    """Host maps of part p as numpy int32 arrays (see include/difvm.h)."""
    info = difvm_partition_info(part, p)
    n = info["n_parts"]
    out = dict(cell_global=np.empty(info["n_owned"] + info["n_ghost"], np.int32),
               face_global=np.empty(info["n_internal_faces"], np.int32),
               bface_global=np.empty(info["n_boundary_faces"], np.int32),
               recv_start=np.empty(n + 1, np.int32), send_start=np.empty(n + 1, np.int32),
               send_cells=np.empty(info["n_send"], np.int32))
    _check(lib().difvm_partition_maps(part, int(p), *[a.ctypes.data_as(_i32p) for a in out.values()]),
           "difvm_partition_maps")
    return out


def difvm_mesh_create_part(ctx, part, p):
    out = _vp()
    _check(lib().difvm_mesh_create_part(ctx, part, int(p), C.byref(out)), "difvm_mesh_create_part")
    return out


def difvm_halo_pack(m, ncomp, x, send_buf):
    return _check(lib().difvm_halo_pack(m, _dtype_code(x), int(ncomp), _ptr(x), _ptr(send_buf)), "difvm_halo_pack")


def difvm_halo_unpack(m, ncomp, recv_buf, x):
    return _check(lib().difvm_halo_unpack(m, _dtype_code(x), int(ncomp), _ptr(recv_buf), _ptr(x)),
                  "difvm_halo_unpack")


def difvm_mesh_set_launch(m, knob, value):
    _check(lib().difvm_mesh_set_launch(m, int(knob), int(value)), "difvm_mesh_set_launch")


def difvm_mesh_get_launch(m, knob):
    v = C.c_int32(0)
    _check(lib().difvm_mesh_get_launch(m, int(knob), C.byref(v)), "difvm_mesh_get_launch")
    return v.value


def difvm_tune(m, cache_path=None):
    """Autotunes the mesh's launch knobs (cache_path: JSON cache file or None); returns knobs timed."""
    n = C.c_int32(0)
    path = None if cache_path is None else str(cache_path).encode()
    _check(lib().difvm_tune(m, path, C.byref(n)), "difvm_tune")
    return n.value


def difvm_mesh_get_info(m):
    info = MeshInfo()
    _check(lib().difvm_mesh_get_info(m, C.byref(info)), "difvm_mesh_get_info")
    return {n: getattr(info, n) for n, _ in MeshInfo._fields_}


def difvm_mesh_destroy(m):
    _check(lib().difvm_mesh_destroy(m), "difvm_mesh_destroy")


def difvm_permute(m, ncomp, kind, direction, src, dst):
    return _check(lib().difvm_permute(m, _dtype_code(src), int(ncomp), int(kind), int(direction), _ptr(src), _ptr(dst)),
                  "difvm_permute")


def difvm_op_interp(m, ncomp, bc, phi, phi_b, phi_f):
    return _check(lib().difvm_op_interp(m, _dtype_code(phi), ncomp, bc, _ptr(phi), _ptr(phi_b), _ptr(phi_f)),
                  "difvm_op_interp")


def difvm_op_grad(m, ncomp, bc, phi, phi_b, grad):
    return _check(lib().difvm_op_grad(m, _dtype_code(phi), ncomp, bc, _ptr(phi), _ptr(phi_b), _ptr(grad)),
                  "difvm_op_grad")


def difvm_op_deferred_correction(m, conv, ncomp, flux, phi, grad, out):
    return _check(lib().difvm_op_deferred_correction(m, _dtype_code(out), CONV[conv] if isinstance(conv, str) else conv,
                                                     ncomp, _ptr(flux), _ptr(phi), _ptr(grad), _ptr(out)),
                  "difvm_op_deferred_correction")


def difvm_op_div(m, scheme, ncomp, bc, flux, psi, psi_b, out):
    return _check(lib().difvm_op_div(m, _dtype_code(flux), scheme, ncomp, bc, _ptr(flux), _ptr(psi), _ptr(psi_b),
                                     _ptr(out)), "difvm_op_div")


def difvm_op_laplacian(m, bc, gamma_f, phi, grad_phi, phi_b, out):
    return _check(lib().difvm_op_laplacian(m, _dtype_code(phi), bc, _ptr(gamma_f), _ptr(phi), _ptr(grad_phi),
                                           _ptr(phi_b), _ptr(out)), "difvm_op_laplacian")


def ldu(diag, upper, lower=None):
    """difvm_ldu over device tensors; the returned struct keeps the tensors alive."""
    A = Ldu(_dtype_code(diag), _ptr(diag), _ptr(upper), _ptr(lower))
    A._keep = (diag, upper, lower)
    return A


def difvm_ldu_spmv(m, ncomp, transpose, A, x, y):
    return _check(lib().difvm_ldu_spmv(m, ncomp, int(transpose), C.byref(A), _ptr(x), _ptr(y)), "difvm_ldu_spmv")


def difvm_ldu_assemble_laplace(m, bc, gamma_f, phi_b, A, rhs_bc):
    return _check(lib().difvm_ldu_assemble_laplace(m, bc, _ptr(gamma_f), _ptr(phi_b), C.byref(A), _ptr(rhs_bc)),
                  "difvm_ldu_assemble_laplace")


def difvm_ldu_assemble_momentum(m, nu, dt, flux, U, U_b, A, b):
    return _check(lib().difvm_ldu_assemble_momentum(m, float(nu), float(dt), _ptr(flux), _ptr(U), _ptr(U_b),
                                                    C.byref(A), _ptr(b)), "difvm_ldu_assemble_momentum")


def difvm_ldu_assemble_momentum_noalloc(m, nu, dt, flux, U, U_b, A, b):
    return _check(lib().difvm_ldu_assemble_momentum_noalloc(m, float(nu), float(dt), _ptr(flux), _ptr(U), _ptr(U_b),
                                                            C.byref(A), _ptr(b)), "difvm_ldu_assemble_momentum_noalloc")


NOALLOC_MAX_CELLS = 131072  # DIFVM_NOALLOC_MAX_CELLS of include/difvm.h


def difvm_solve_pcg(m, A, b, x, tol, maxit):
    st = SolveStats()
    status = _check(lib().difvm_solve_pcg(m, C.byref(A), _ptr(b), _ptr(x), float(tol), int(maxit), C.byref(st)),
                    "difvm_solve_pcg")
    return status, st.iters[0], st.residual[0]


def difvm_amg_create(m, A):
    out = _vp()
    _check(lib().difvm_amg_create(m, C.byref(A), C.byref(out)), "difvm_amg_create")
    return out


def difvm_amg_setup_host(ptr, col, val, diag):
    """host-only hierarchy of a symmetric CSR matrix (off-diagonals) with diagonal diag: returns (agg, rows)"""
    n = len(diag)
    ptr = np.ascontiguousarray(ptr, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.float64)
    diag = np.ascontiguousarray(diag, np.float64)
    agg = np.empty(n, np.int32)
    rows = np.zeros(64, np.int32)
    nl = C.c_int32(0)
    _check(lib().difvm_amg_setup_host(n, ptr.ctypes.data_as(_i32p), col.ctypes.data_as(_i32p), val.ctypes.data_as(_f64p),
                                      diag.ctypes.data_as(_f64p), agg.ctypes.data_as(_i32p), rows.ctypes.data_as(_i32p),
                                      64, C.byref(nl)), "difvm_amg_setup_host")
    return agg, rows[:nl.value].tolist()


def difvm_amg_destroy(a):
    _check(lib().difvm_amg_destroy(a), "difvm_amg_destroy")


def difvm_amg_levels(a):
    rows = np.zeros(64, np.int32)
    n = C.c_int32(0)
    _check(lib().difvm_amg_levels(a, rows.ctypes.data_as(_i32p), 64, C.byref(n)), "difvm_amg_levels")
    return rows[:n.value].tolist()


def difvm_amg_apply(a, r, z):
    _check(lib().difvm_amg_apply(a, _ptr(r), _ptr(z)), "difvm_amg_apply")


def difvm_solve_pcg_amg(a, A, b, x, tol, maxit):
    st = SolveStats()
    status = _check(lib().difvm_solve_pcg_amg(a, C.byref(A), _ptr(b), _ptr(x), float(tol), int(maxit), C.byref(st)),
                    "difvm_solve_pcg_amg")
    return status, st.iters[0], st.residual[0]


def difvm_piso_rebuild_preconditioner(p):
    _check(lib().difvm_piso_rebuild_preconditioner(p), "difvm_piso_rebuild_preconditioner")


def difvm_solve_bicgstab(m, A, ncomp, b, x, tol, maxit):
    st = SolveStats()
    status = _check(lib().difvm_solve_bicgstab(m, C.byref(A), ncomp, _ptr(b), _ptr(x), float(tol), int(maxit),
                                               C.byref(st)), "difvm_solve_bicgstab")
    return status, list(st.iters)[:ncomp], list(st.residual)[:ncomp]


def piso_params(nu, dt, n_corr=2, tol_p=1e-8, tol_u=1e-8, maxit_p=2000, maxit_u=500, p_ref_cell=0, p_ref_value=0.0,
                conv="upwind", time="backward_euler", precond="jacobi"):
    return PisoParams(C.sizeof(PisoParams), nu, dt, n_corr, tol_p, tol_u, maxit_p, maxit_u, p_ref_cell, p_ref_value,
                      CONV[conv], TIME[time], PRECOND[precond])


def difvm_piso_create(m, params):
    out = _vp()
    _check(lib().difvm_piso_create(m, C.byref(params), C.byref(out)), "difvm_piso_create")
    return out


def difvm_piso_destroy(p):
    _check(lib().difvm_piso_destroy(p), "difvm_piso_destroy")


def difvm_piso_set_boundary(p, U_b, p_b):
    _check(lib().difvm_piso_set_boundary(p, _ptr(U_b), _ptr(p_b)), "difvm_piso_set_boundary")


def difvm_piso_set_windkessel(p, wid, Rp, Cc, Rd, pc):
    _check(lib().difvm_piso_set_windkessel(p, int(wid), float(Rp), float(Cc), float(Rd), float(pc)),
           "difvm_piso_set_windkessel")


def difvm_piso_set_viscosity(p, nu_seg):
    nu = np.ascontiguousarray(nu_seg, dtype=np.float64)
    _check(lib().difvm_piso_set_viscosity(p, int(nu.size), nu.ctypes.data_as(_f64p)), "difvm_piso_set_viscosity")


def _stats_arrays(stats, n_corr):
    it = np.array([[*s.it_u, *list(s.it_p)[:n_corr]] for s in stats], dtype=np.int32)
    res = np.array([[*s.res_u, *list(s.res_p)[:n_corr]] for s in stats])
    return it, res


def difvm_piso_segment_stats(p, n_seg, n_corr=2):
    """Per-segment (iterations, residuals, status) of the most recent step."""
    stats = (StepStats * n_seg)()
    _check(lib().difvm_piso_segment_stats(p, int(n_seg), stats), "difvm_piso_segment_stats")
    it, res = _stats_arrays(stats, n_corr)
    return it, res, np.array([s.status for s in stats], dtype=np.int32)


def difvm_piso_transport_scalar(p, D, bc, c_b, c):
    """One passive-scalar step in place on c (device, user order); returns (status, iters, residual)."""
    st = SolveStats()
    status = _check(lib().difvm_piso_transport_scalar(p, float(D), int(bc), _ptr(c_b), _ptr(c), C.byref(st)),
                    "difvm_piso_transport_scalar")
    return status, st.iters[0], st.residual[0]


def difvm_piso_set_graph(p, enable, extra_iters=16):
    _check(lib().difvm_piso_set_graph(p, int(enable), int(extra_iters)), "difvm_piso_set_graph")


def difvm_piso_graph_info(p):
    """(replays, redos, captures) of graph mode."""
    v = [C.c_int64(0) for _ in range(3)]
    _check(lib().difvm_piso_graph_info(p, *[C.byref(x) for x in v]), "difvm_piso_graph_info")
    return tuple(x.value for x in v)


def difvm_piso_set_state(p, U, pres, phi):
    _check(lib().difvm_piso_set_state(p, _ptr(U), _ptr(pres), _ptr(phi)), "difvm_piso_set_state")


def difvm_piso_get_state(p, U, pres, phi, n_wk=0):
    pc = (C.c_double * max(1, n_wk))()
    _check(lib().difvm_piso_get_state(p, _ptr(U), _ptr(pres), _ptr(phi), pc), "difvm_piso_get_state")
    return np.array(pc[:n_wk])


def difvm_piso_step(p, nsteps, n_corr=2):
    stats = (StepStats * max(1, nsteps))()
    status = _check(lib().difvm_piso_step(p, int(nsteps), stats), "difvm_piso_step")
    it, res = _stats_arrays(stats[:nsteps], n_corr)
    return status, it, res


def difvm_piso_precond_info(p):
    """(rows per level, finest first; algorithmic bytes of one V-cycle) of the AMG preconditioner."""
    n = C.c_int32()
    rows = (C.c_int32 * 64)()
    vb = C.c_double()
    _check(lib().difvm_piso_precond_info(p, C.byref(n), rows, 64, C.byref(vb)), "difvm_piso_precond_info")
    return [rows[k] for k in range(min(n.value, 64))], vb.value


def difvm_piso_step_trace(p, U_star, p_corr, n_corr=2):
    """One step that also writes the predictor's solution U_star[Nc, 3] and each corrector's pressure
    p_corr[n_corr, Nc] (device tensors, user order).  Returns (status, iters[3+n_corr], res)."""
    st = StepStats()
    status = _check(lib().difvm_piso_step_trace(p, _ptr(U_star), _ptr(p_corr), C.byref(st)), "difvm_piso_step_trace")
    it, res = _stats_arrays([st], n_corr)
    return status, it[0], res[0]


def difvm_tape_create(p, nsteps, ckpt_every):
    out = _vp()
    _check(lib().difvm_tape_create(p, int(nsteps), int(ckpt_every), C.byref(out)), "difvm_tape_create")
    return out


def difvm_tape_destroy(t):
    _check(lib().difvm_tape_destroy(t), "difvm_tape_destroy")


def difvm_piso_forward_record(p, t, nsteps, n_corr=2):
    stats = (StepStats * max(1, nsteps))()
    status = _check(lib().difvm_piso_forward_record(p, t, stats), "difvm_piso_forward_record")
    it = np.array([[*s.it_u, *list(s.it_p)[:n_corr]] for s in stats[:nsteps]], dtype=np.int32)
    return status, it


def difvm_tape_boundary_cotangent(t, gU_b):
    return _check(lib().difvm_tape_boundary_cotangent(t, _ptr(gU_b)), "difvm_tape_boundary_cotangent")


def difvm_tape_set_graph(t, enable=True, extra_iters=16):
    _check(lib().difvm_tape_set_graph(t, int(bool(enable)), int(extra_iters)), "difvm_tape_set_graph")


def difvm_tape_graph_info(t):
    """(replays, redos, captures) of the tape's graph mode."""
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().difvm_tape_graph_info(t, C.byref(a), C.byref(b), C.byref(c)), "difvm_tape_graph_info")
    return a.value, b.value, c.value


def difvm_piso_adjoint(p, t, gU_N, gp_N, gphi_N, gpc_N, adj_tol, gU_0, gp_0, gphi_0, n_wk):
    """Returns (status, gpc_0[n_wk], gwk[n_wk, 3]); device outputs are written in place."""
    gpc_in = None
    if gpc_N is not None and n_wk:
        gpc_in = (C.c_double * n_wk)(*[float(v) for v in gpc_N])
    gpc_out = (C.c_double * max(1, n_wk))()
    gwk = (C.c_double * max(1, 3 * n_wk))()
    status = _check(lib().difvm_piso_adjoint(p, t, _ptr(gU_N), _ptr(gp_N), _ptr(gphi_N), gpc_in, float(adj_tol),
                                             _ptr(gU_0), _ptr(gp_0), _ptr(gphi_0), gpc_out, gwk), "difvm_piso_adjoint")
    return status, np.array(gpc_out[:n_wk]), np.array(gwk[:3 * n_wk]).reshape(n_wk, 3)


# ------------------------------------------------------------------------------------------------
# owning handles
# ------------------------------------------------------------------------------------------------
class Context:
    """A library context on one device and stream.  torch_allocator=True (default) routes every device
    allocation of the library through torch's caching allocator (difvm_ctx_set_allocator)."""

    def __init__(self, device=0, stream=None, torch_allocator=True):
        import torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.h = difvm_ctx_create(device, C.c_void_p(stream.cuda_stream))
        self.allocator = None
        if torch_allocator:
            self.allocator = TorchAllocator(device)
            difvm_ctx_set_allocator(self.h, self.allocator.alloc_fn, self.allocator.free_fn)

    def close(self):
        if self.h:
            difvm_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    """A mesh uploaded to the device (internal order).  Keeps the meshgen.Mesh for user-order sizes.
    flags=None: RCM order and the correction scheme named by mesh.meta["nonorth"] (over-relaxed if
    absent)."""

    def __init__(self, ctx, mesh, flags=None, seg_cell_start=None):
        self.ctx = ctx
        self.src = mesh
        if flags is None:
            flags = RENUMBER_RCM | NONORTH[mesh.meta.get("nonorth", "overrelaxed")]
        if seg_cell_start is None:
            self.h = difvm_mesh_create(ctx.h, mesh, flags)
        else:
            self.h = difvm_mesh_create_segments(ctx.h, mesh, seg_cell_start, flags)
        self.info = difvm_mesh_get_info(self.h)

    def close(self):
        if self.h:
            difvm_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def to_internal(self, t, kind, ncomp=None):
        import torch
        ncomp = ncomp if ncomp is not None else (1 if t.dim() == 1 else int(np.prod(t.shape[1:])))
        out = torch.empty_like(t)
        difvm_permute(self.h, ncomp, kind, TO_INTERNAL, t.contiguous(), out)
        return out

    def to_user(self, t, kind, ncomp=None):
        import torch
        ncomp = ncomp if ncomp is not None else (1 if t.dim() == 1 else int(np.prod(t.shape[1:])))
        out = torch.empty_like(t)
        difvm_permute(self.h, ncomp, kind, FROM_INTERNAL, t.contiguous(), out)
        return out


class Partition:
    """Slab partition of a meshgen.Mesh for a halo exchange (host only): per part its info dict and
    host maps (difvm_partition_info / difvm_partition_maps)."""

    def __init__(self, mesh, n_parts, flags=None):
        if flags is None:
            flags = RENUMBER_RCM | NONORTH[mesh.meta.get("nonorth", "overrelaxed")]
        self.src = mesh
        self.n_parts = int(n_parts)
        self.h = difvm_partition_create(mesh, n_parts, flags)
        self.info = [difvm_partition_info(self.h, p) for p in range(self.n_parts)]
        self.maps = [difvm_partition_maps(self.h, p) for p in range(self.n_parts)]

    def close(self):
        if self.h:
            difvm_partition_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PartMesh:
    """Part p of a Partition uploaded to the device (local order: owned cells, then ghosts)."""

    def __init__(self, ctx, partition, p):
        self.ctx = ctx
        self.p = int(p)
        self.part = partition.info[p]
        self.maps = partition.maps[p]
        self.h = difvm_mesh_create_part(ctx.h, partition.h, p)
        self.info = difvm_mesh_get_info(self.h)

    def pack(self, x, send_buf):
        ncomp = 1 if x.dim() == 1 else int(np.prod(x.shape[1:]))
        difvm_halo_pack(self.h, ncomp, x, send_buf)

    def unpack(self, recv_buf, x):
        ncomp = 1 if x.dim() == 1 else int(np.prod(x.shape[1:]))
        difvm_halo_unpack(self.h, ncomp, recv_buf, x)

    def close(self):
        if self.h:
            difvm_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Piso:
    def __init__(self, mesh, params):
        self.mesh = mesh
        self.params = params
        self.h = difvm_piso_create(mesh.h, params)

    def close(self):
        if self.h:
            difvm_piso_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_boundary(self, U_b=None, p_b=None):
        difvm_piso_set_boundary(self.h, U_b, p_b)

    def set_windkessel(self, wid, Rp, Cc, Rd, pc):
        difvm_piso_set_windkessel(self.h, wid, Rp, Cc, Rd, pc)

    def transport_scalar(self, D, bc, c_b, c):
        return difvm_piso_transport_scalar(self.h, D, bc, c_b, c)

    def set_graph(self, enable=True, extra_iters=16):
        difvm_piso_set_graph(self.h, enable, extra_iters)

    def graph_info(self):
        return difvm_piso_graph_info(self.h)

    def set_viscosity(self, nu_seg):
        difvm_piso_set_viscosity(self.h, nu_seg)

    def segment_stats(self):
        return difvm_piso_segment_stats(self.h, self.mesh.info["n_segments"], self.params.n_corr)

    def set_state(self, U, p, phi=None):
        difvm_piso_set_state(self.h, U, p, phi)

    def get_state(self):
        import torch
        src = self.mesh.src
        dev = self.mesh.ctx.device
        U = torch.empty((src.n_cells, 3), dtype=torch.float64, device=dev)
        p = torch.empty(src.n_cells, dtype=torch.float64, device=dev)
        phi = torch.empty(src.n_faces, dtype=torch.float64, device=dev)
        pc = difvm_piso_get_state(self.h, U, p, phi, self.mesh.info["n_windkessel"])
        return U, p, phi, pc

    def step(self, nsteps=1):
        return difvm_piso_step(self.h, nsteps, self.params.n_corr)

    def step_trace(self):
        """One step; returns (status, iters, res, U_star[Nc, 3], p_corr[n_corr, Nc]) with the solution of
        each linear solve of the step (device tensors, user order)."""
        import torch
        src = self.mesh.src
        dev = self.mesh.ctx.device
        Us = torch.empty((src.n_cells, 3), dtype=torch.float64, device=dev)
        pc = torch.empty((self.params.n_corr, src.n_cells), dtype=torch.float64, device=dev)
        status, it, res = difvm_piso_step_trace(self.h, Us, pc, self.params.n_corr)
        return status, it, res, Us, pc
