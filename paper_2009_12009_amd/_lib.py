"""ctypes binding of libamrmg.so: struct layouts, the C entry points and errors.

Only argument marshalling lives here; every step of the solve runs in the HIP
library.  Importing this module loads the library and fails loudly if it has
not been built.
"""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamrmg.so")

MG_OK = 0
MG_ERR_ARG = -1
MG_ERR_INVALID_BOXARRAY = -2
MG_ERR_MISMATCH = -3
MG_ERR_WORKSPACE = -4
MG_ERR_HIP = -5
MG_ERR_NAN = -6
MG_ERR_DIVERGED = -7
MG_ERR_NOT_CONVERGED = -8
MG_ERR_SINGULAR = -9
STATUS_NAMES = {v: k for k, v in dict(globals()).items() if k.startswith("MG_ERR_") or k == "MG_OK"}

MG_BC_PERIODIC = 0
MG_BC_DIRICHLET0 = 1
MG_F64 = 0
MG_F32 = 1
MG_PREC_F64 = 0
MG_PREC_F32_REFINE = 1

# profiling families (mg_kernel_stats)
(FAM_SMOOTH, FAM_RESID, FAM_EXCHANGE, FAM_RESTRICT, FAM_PROLONG, FAM_COARSE, FAM_UPDATE,
 FAM_RIM) = range(8)


class MgBox(C.Structure):
    _fields_ = [("lo", C.c_int32 * 3), ("hi", C.c_int32 * 3)]


class MgGeom(C.Structure):
    _fields_ = [("domain", MgBox), ("prob_lo", C.c_double * 3), ("prob_hi", C.c_double * 3),
                ("is_periodic", C.c_int32 * 3)]


class MgMultiFab(C.Structure):
    _fields_ = [("nbox", C.c_int32), ("boxes", C.POINTER(MgBox)), ("ngrow", C.c_int32),
                ("ncomp", C.c_int32), ("ixtype", C.c_int32 * 3), ("dtype", C.c_int32),
                ("data", C.c_void_p), ("offsets", C.POINTER(C.c_int64))]


class MgOpts(C.Structure):
    _fields_ = [("nu1", C.c_int32), ("nu2", C.c_int32), ("max_iter", C.c_int32),
                ("bottom_max_iter", C.c_int32), ("min_bottom_edge", C.c_int32),
                ("precision", C.c_int32), ("use_graph", C.c_int32), ("tune", C.c_int32),
                ("verbose", C.c_int32), ("aggregate", C.c_int32), ("bottom_rel_tol", C.c_double),
                ("fused_min_edge", C.c_int32), ("krylov", C.c_int32),
                ("ghost_write", C.c_int32), ("interp_fold", C.c_int32),
                ("bottom_solver", C.c_int32), ("restrict_fold", C.c_int32),
                ("stop_fold", C.c_int32), ("coarse_tail", C.c_int32)]


class MgInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("nlevels", C.c_int32), ("bottom_iters", C.c_int32),
                ("converged", C.c_int32), ("rel_resid", C.c_double), ("abs_resid", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("tail_level", C.c_int32)]


class MgCopyTag(C.Structure):
    _fields_ = [("dst", C.c_int32), ("src", C.c_int32), ("dst_region", MgBox),
                ("shift", C.c_int32 * 3)]


# name -> (restype, argtypes)
P = C.POINTER
SIGNATURES = {
    "mg_default_opts": (None, [P(MgOpts)]),
    "mg_query_workspace": (C.c_int, [P(MgBox), C.c_int32, P(MgGeom), P(MgOpts), C.c_int32,
                                     P(C.c_size_t)]),
    "mg_create": (C.c_int, [P(MgBox), C.c_int32, P(MgGeom), P(C.c_int32), P(C.c_int32),
                            C.c_double, C.c_double, P(MgMultiFab), P(P(MgMultiFab)), P(MgOpts),
                            C.c_void_p, C.c_size_t, C.c_void_p, P(C.c_void_p)]),
    "mg_set_coefficients": (C.c_int, [C.c_void_p, P(MgMultiFab), P(P(MgMultiFab))]),
    "mg_set_coefficients_global": (C.c_int, [C.c_void_p, C.c_void_p, P(C.c_void_p), C.c_int32]),
    "mg_solve": (C.c_int, [C.c_void_p, P(MgMultiFab), P(MgMultiFab), C.c_double, C.c_double,
                           P(MgInfo), P(C.c_double)]),
    "mg_apply": (C.c_int, [C.c_void_p, P(MgMultiFab), P(MgMultiFab)]),
    "mg_face_grad_logb": (C.c_int, [C.c_void_p, P(MgMultiFab), P(MgMultiFab), P(P(MgMultiFab))]),
    "mg_face_grad_logb_global": (C.c_int, [C.c_void_p, P(MgMultiFab), P(MgMultiFab),
                                           P(C.c_void_p)]),
    "mg_copy_valid": (C.c_int, [C.c_void_p, P(MgMultiFab), P(MgMultiFab)]),
    "mg_destroy": (None, [C.c_void_p]),
    "fill_boundary": (C.c_int, [P(MgMultiFab), P(MgGeom), C.c_void_p]),
    "mg_fill_boundary": (C.c_int, [P(MgMultiFab), P(MgGeom), C.c_void_p]),
    "mg_fill_boundary_noalloc": (C.c_int, [P(MgMultiFab), P(MgGeom), C.c_void_p]),
    "mg_copy_tags": (C.c_int, [P(MgBox), C.c_int32, P(MgGeom), C.c_int32, P(MgCopyTag),
                               C.c_int32, P(C.c_int32)]),
    "mg_num_levels": (C.c_int, [P(MgBox), C.c_int32, P(MgGeom), P(MgOpts), P(C.c_int32)]),
    "mg_profile": (C.c_int, [C.c_void_p, C.c_int32]),
    "mg_kernel_stats": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_double), P(C.c_int64)]),
    "mg_time_smoother": (C.c_int, [C.c_void_p, P(MgMultiFab), P(MgMultiFab), C.c_int32,
                                   P(C.c_double)]),
    "mg_stream_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "mg_get_tile_shape": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_int32)]),
    "mg_set_class_tile_shape": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                          C.c_int32]),
    "mg_get_class_tile_shapes": (C.c_int, [C.c_void_p, P(C.c_int32), C.c_int32, P(C.c_int32)]),
    "mg_set_tile_shape": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                    C.c_int32]),
    "mg_query_workspace_amr": (C.c_int, [P(MgBox), C.c_int32, P(MgBox), C.c_int32, P(MgGeom),
                                         P(MgOpts), P(C.c_size_t)]),
    "mg_create_amr": (C.c_int, [P(MgBox), C.c_int32, P(MgBox), C.c_int32, P(MgGeom), C.c_double,
                                C.c_double, P(P(MgMultiFab)), P(P(MgMultiFab)), P(MgOpts),
                                C.c_void_p, C.c_size_t, C.c_void_p, P(C.c_void_p)]),
    "mg_solve_amr": (C.c_int, [C.c_void_p, P(MgMultiFab), P(MgMultiFab), P(MgMultiFab),
                               P(MgMultiFab), C.c_double, C.c_double, P(MgInfo), P(C.c_double)]),
    "mg_nodal_query_workspace": (C.c_int, [P(MgBox), C.c_int32, P(MgGeom), P(MgOpts),
                                           P(C.c_size_t)]),
    "mg_nodal_create": (C.c_int, [P(MgBox), C.c_int32, P(MgGeom), P(C.c_int32), P(C.c_int32),
                                  P(MgMultiFab), P(MgOpts), C.c_void_p, C.c_size_t, C.c_void_p,
                                  P(C.c_void_p)]),
    "mg_nodal_solve": (C.c_int, [C.c_void_p, P(MgMultiFab), P(MgMultiFab), C.c_double,
                                 C.c_double, P(MgInfo), P(C.c_double)]),
    "mg_nodal_apply": (C.c_int, [C.c_void_p, P(MgMultiFab), P(MgMultiFab)]),
    "mg_nodal_num_levels": (C.c_int, [C.c_void_p, P(C.c_int32)]),
    "mg_nodal_time_smoother": (C.c_int, [C.c_void_p, C.c_int32, P(C.c_double)]),
    "mg_nodal_destroy": (None, [C.c_void_p]),
    "mg_release_caches": (None, []),
    "mg_last_error": (C.c_char_p, []),
}


class MGError(RuntimeError):
    def __init__(self, code, where, msg):
        self.code = code
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2009_12009_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def check(code, where):
    if code != MG_OK:
        raise MGError(code, where, lib.mg_last_error().decode())
    return code


def boxes_array(boxes):
    arr = (MgBox * len(boxes))()
    for i, (lo, hi) in enumerate(boxes):
        arr[i].lo[:] = [int(x) for x in lo]
        arr[i].hi[:] = [int(x) for x in hi]
    return arr


def geom_struct(domain, periodic, prob_lo=(0.0, 0.0, 0.0), prob_hi=(1.0, 1.0, 1.0)):
    g = MgGeom()
    g.domain.lo[:] = [int(x) for x in domain[0]]
    g.domain.hi[:] = [int(x) for x in domain[1]]
    g.prob_lo[:] = [float(x) for x in prob_lo]
    g.prob_hi[:] = [float(x) for x in prob_hi]
    g.is_periodic[:] = [1 if p else 0 for p in periodic]
    return g


def default_opts(**kw):
    o = MgOpts()
    lib.mg_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o
