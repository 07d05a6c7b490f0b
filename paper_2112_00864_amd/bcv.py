"""ctypes binding of libbcvol (include/bcv.h): argument marshalling only.

Every computation runs in the library's HIP kernels; PyTorch supplies device memory and
streams. The binding raises if the library has not been built.
"""

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbcvol.so")
_lib = None

OK, EINVAL, ENOMEM, EDEVICE, ENOTSUP, ESTATE = range(6)
NEAR_QUADRATURE, NEAR_ASSEMBLED = 0, 1
MARK_FACE, MARK_NEIGHBOR = 0, 1
FP64, MIXED_F32, MIXED_SPLIT16 = 0, 1, 2
PART_NEAR, PART_FAR = 1, 2
TOUCH_CLASSES = ("self", "face", "edge", "vertex", "face2", "edge2", "vertex2")


class BCVError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("bcv status %d: %s" % (status, message))
        self.status = status


GEOM_BOX, GEOM_BALL = 0, 1


class MeshDesc(ctypes.Structure):
    _fields_ = [("geometry", ctypes.c_int), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("L", ctypes.c_int), ("marking", ctypes.c_int)]


def _mesh_desc(L, marking, lo=None, hi=None, geometry=GEOM_BOX):
    d = MeshDesc()
    d.geometry, d.L, d.marking = int(geometry), int(L), int(marking)
    for ax in range(3):
        d.lo[ax] = 0.0 if lo is None else float(lo[ax])
        d.hi[ax] = 0.0 if hi is None else float(hi[ax])
    return d


class PlanOpts(ctypes.Structure):
    _fields_ = [("eta0", ctypes.c_double), ("q", ctypes.c_int), ("precision", ctypes.c_int),
                ("direct", ctypes.c_int), ("nearfield", ctypes.c_int), ("streams", ctypes.c_int),
                ("surrogate", ctypes.c_void_p), ("surrogate_tol", ctypes.c_double), ("near_unit", ctypes.c_int),
                ("m2l_max_slots", ctypes.c_int), ("q_schedule", ctypes.c_int), ("near_order", ctypes.c_int),
                ("boundary", ctypes.c_int), ("basis_degree", ctypes.c_int), ("exact_moments", ctypes.c_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("n_leaves", "n_cells", "n_near", "n_touch", "n_m2l", "n_m2l_lanes",
                                              "n_offsets", "n_m2l_read_lanes", "n_faces", "n_btv_near",
                                              "n_btv_touch", "n_vtb_near", "n_near_ordered",
                                              "device_bytes")] + [
        ("K", ctypes.c_int32), ("L", ctypes.c_int32), ("surrogate_classes", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("n_dofs", ctypes.c_int64), ("n_basis_vals", ctypes.c_int64), ("n_basis_cols", ctypes.c_int64),
        ("n_btv_m2l", ctypes.c_int64), ("n_vtb_m2l", ctypes.c_int64), ("n_mapped_touch_pairs", ctypes.c_int64)]


CONTACT_FACE, CONTACT_EDGE, CONTACT_VERTEX = 1, 2, 3


class TouchPair(ctypes.Structure):
    _fields_ = [("contact", ctypes.c_int32), ("pad", ctypes.c_int32), ("rho", ctypes.c_double),
                ("off", ctypes.c_double * 2)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("n_train", ctypes.c_int64), ("n_valid", ctypes.c_int64), ("epochs", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("lr", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("n_gauss_lo", ctypes.c_int32), ("n_gauss_hi", ctypes.c_int32), ("tol", ctypes.c_double)]


class TrainReport(ctypes.Structure):
    _fields_ = [("residual_scale", ctypes.c_double), ("kappa", ctypes.c_double), ("valid_max_rel_err_lo", ctypes.c_double),
                ("valid_max_rel_err", ctypes.c_double), ("valid_rms_rel_err", ctypes.c_double),
                ("valid_max_rel_err_accepted", ctypes.c_double), ("valid_accepted", ctypes.c_int64),
                ("valid_reported", ctypes.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("libbcvol.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(_LIB_PATH)
        vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
        L.bcv_build_bc_tree.argtypes = [ctypes.POINTER(MeshDesc), ctypes.POINTER(vp)]
        L.bcv_tree_num_leaves.argtypes = [vp, i64p]
        L.bcv_tree_leaves.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
        L.bcv_vtv_apply_batched.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                            vp]
        L.bcv_tree_destroy.argtypes = [vp]
        L.bcv_tree_destroy.restype = None
        L.bcv_plan_interactions.argtypes = [vp, ctypes.POINTER(PlanOpts), ctypes.c_int, ctypes.POINTER(vp)]
        L.bcv_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.bcv_plan_destroy.argtypes = [vp]
        L.bcv_plan_destroy.restype = None
        L.bcv_vtv_apply.argtypes = [vp, vp, vp, vp]
        L.bcv_vtv_apply_parts.argtypes = [vp, vp, vp, vp, ctypes.c_int]
        L.bcv_vtb_apply.argtypes = [vp, vp, vp, vp]
        L.bcv_btv_apply.argtypes = [vp, vp, vp, vp, vp]
        L.bcv_tree_num_faces.argtypes = [vp, i64p]
        L.bcv_tree_faces.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.bcv_boundary_touching_integrals.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.bcv_plan_enable_timing.argtypes = [vp, ctypes.c_int]
        L.bcv_plan_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i64p]
        L.bcv_touching_integrals.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.bcv_touching_basis_block.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        dp, fp, i32p = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int32)
        L.bcv_box_pair_integrals.argtypes = [ctypes.c_int, ctypes.c_int64, dp, ctypes.c_int, dp]
        L.bcv_touch_pair_quadrature.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.POINTER(TouchPair), ctypes.c_int,
                                                dp]
        L.bcv_mlp_create.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(vp)]
        L.bcv_mlp_destroy.argtypes = [vp]
        L.bcv_mlp_destroy.restype = None
        L.bcv_mlp_num_params.argtypes = [vp, i64p]
        L.bcv_mlp_get_params.argtypes = [vp, fp]
        L.bcv_mlp_set_params.argtypes = [vp, fp]
        L.bcv_mlp_forward.argtypes = [vp, ctypes.c_int64, fp, fp]
        L.bcv_mlp_forward_noalloc.argtypes = [vp, ctypes.c_int64, vp, vp, vp]
        L.bcv_mlp_loss_grad.argtypes = [vp, ctypes.c_int64, fp, fp, dp, fp]
        L.bcv_mlp_train.argtypes = [vp, ctypes.POINTER(TrainOpts), ctypes.POINTER(TrainReport)]
        L.bcv_surrogate_eval.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(TouchPair), ctypes.c_double, dp, dp,
                                         i32p, i64p]
        L.bcv_mapped_pair_entries.argtypes = [ctypes.c_int, ctypes.c_int64, dp, dp, dp]
        L.bcv_mlp_save.argtypes = [vp, ctypes.c_char_p]
        L.bcv_mlp_load.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(vp)]
        L.bcv_build_bc_forest.argtypes = [ctypes.c_int, ctypes.POINTER(MeshDesc), ctypes.POINTER(vp)]
        L.bcv_tree_leaf_mesh.argtypes = [vp, i32p]
        L.bcv_vtv_graph_create.argtypes = [vp, vp, vp, ctypes.POINTER(vp)]
        L.bcv_graph_launch.argtypes = [vp, vp]
        L.bcv_graph_destroy.argtypes = [vp]
        L.bcv_graph_destroy.restype = None
        L.bcv_autotune.argtypes = [vp, ctypes.POINTER(PlanOpts), ctypes.c_int, ctypes.c_int, ctypes.POINTER(PlanOpts),
                                   dp]
        L.bcv_last_error.restype = ctypes.c_char_p
        for name in ("bcv_build_bc_tree", "bcv_tree_num_leaves", "bcv_tree_leaves", "bcv_plan_interactions",
                     "bcv_plan_get_info", "bcv_vtv_apply", "bcv_vtv_apply_batched", "bcv_vtv_apply_parts", "bcv_vtb_apply", "bcv_btv_apply",
                     "bcv_touching_integrals", "bcv_plan_enable_timing", "bcv_plan_phase_times",
                     "bcv_box_pair_integrals", "bcv_touch_pair_quadrature", "bcv_mlp_create", "bcv_mlp_num_params",
                     "bcv_mlp_get_params", "bcv_mlp_set_params", "bcv_mlp_forward", "bcv_mlp_forward_noalloc",
                     "bcv_mlp_loss_grad",
                     "bcv_mlp_train", "bcv_surrogate_eval", "bcv_mlp_save", "bcv_mlp_load", "bcv_build_bc_forest",
                     "bcv_tree_leaf_mesh", "bcv_vtv_graph_create", "bcv_graph_launch", "bcv_autotune",
                     "bcv_mapped_pair_entries"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status):
    if status != OK:
        raise BCVError(status, lib().bcv_last_error().decode())


class Tree:
    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        return self._h

    def num_leaves(self):
        n = ctypes.c_int64()
        _check(lib().bcv_tree_num_leaves(self._h, ctypes.byref(n)))
        return n.value

    def leaf_mesh(self):
        """Mesh index of every leaf, int32 (n,)."""
        out = np.empty(self.num_leaves(), dtype=np.int32)
        _check(lib().bcv_tree_leaf_mesh(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def faces(self):
        """(leaf, axis, side) per boundary face in the library's face order, int32 (n_faces, 3)."""
        n = ctypes.c_int64()
        _check(lib().bcv_tree_num_faces(self._h, ctypes.byref(n)))
        out = np.empty((n.value, 3), dtype=np.int32)
        _check(lib().bcv_tree_faces(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def leaves(self):
        """(level, i, j, k) per leaf in leaf order, int32 (n, 4)."""
        out = np.empty((self.num_leaves(), 4), dtype=np.int32)
        _check(lib().bcv_tree_leaves(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None, None))
        return out

    def gauss_points(self):
        """The 2x2x2 Gauss points of every leaf in physical coordinates, (n, 8, 3), and their weights (n, 8)."""
        n = self.num_leaves()
        xyz = np.empty((n, 8, 3))
        w = np.empty((n, 8))
        _check(lib().bcv_tree_leaves(self._h, None, _dp(xyz), _dp(w)))
        return xyz, w

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.bcv_tree_destroy(self._h)
            self._h = None


def build_bc_forest(Ls, marking=0, boxes=None, geometry=GEOM_BOX):
    """One tree holding len(Ls) meshes; mesh m occupies [4m, 4m+1) x [0,1)^2 (see bcv.h).
    marking, geometry: one value for every mesh, or a list with one per mesh. boxes: None (unit
    cubes) or one (lo, hi) cube per mesh."""
    marks = list(marking) if isinstance(marking, (list, tuple)) else [marking] * len(Ls)
    geoms = list(geometry) if isinstance(geometry, (list, tuple)) else [geometry] * len(Ls)
    if len(marks) != len(Ls) or len(geoms) != len(Ls):
        raise ValueError("one marking and one geometry per mesh")
    boxes = [(None, None)] * len(Ls) if boxes is None else list(boxes)
    descs = (MeshDesc * len(Ls))(*[_mesh_desc(L, mk, lo, hi, gm)
                                   for L, mk, (lo, hi), gm in zip(Ls, marks, boxes, geoms)])
    h = ctypes.c_void_p()
    _check(lib().bcv_build_bc_forest(len(Ls), descs, ctypes.byref(h)))
    return Tree(h)


def build_bc_tree(L, marking=0, lo=None, hi=None, geometry=GEOM_BOX):
    """BC octree of the cube [lo, hi] (default: the unit cube)."""
    desc = _mesh_desc(L, marking, lo, hi, geometry)
    h = ctypes.c_void_p()
    _check(lib().bcv_build_bc_tree(ctypes.byref(desc), ctypes.byref(h)))
    return Tree(h)


class Plan:
    def __init__(self, handle, device):
        self._h = handle
        self.device = device
        info = PlanInfo()
        _check(lib().bcv_plan_get_info(self._h, ctypes.byref(info)))
        self.info = {n: getattr(info, n) for n, _ in PlanInfo._fields_}

    @property
    def handle(self):
        return self._h

    @property
    def n_leaves(self):
        return self.info["n_leaves"]

    @property
    def n_dofs(self):
        """Length of f and u: n_leaves, or the basis coefficients of all leaves (basis_degree=1)."""
        return self.info["n_dofs"]

    def destroy(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.bcv_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        self.destroy()


def _opts(q=6, eta0=0.5, direct=False, nearfield=NEAR_QUADRATURE, streams=2, precision=FP64, surrogate=None,
          surrogate_tol=1e-7, near_unit=0, m2l_max_slots=0, boundary=False, near_order=0, q_schedule=0, basis_degree=0,
          exact_moments=False):
    return PlanOpts(eta0, q, precision, 1 if direct else 0, nearfield, streams,
                    surrogate.handle if surrogate is not None else None, surrogate_tol, near_unit, m2l_max_slots,
                    q_schedule, near_order, 1 if boundary else 0, basis_degree, 1 if exact_moments else 0)


def plan_interactions(tree, q=6, eta0=0.5, direct=False, nearfield=NEAR_QUADRATURE, device=0, streams=2,
                      precision=FP64, surrogate=None, surrogate_tol=1e-7, near_unit=0, m2l_max_slots=0,
                      boundary=False, near_order=0, q_schedule=0, basis_degree=0, exact_moments=False):
    opts = _opts(q, eta0, direct, nearfield, streams, precision, surrogate, surrogate_tol, near_unit, m2l_max_slots,
                 boundary, near_order, q_schedule, basis_degree, exact_moments)
    h = ctypes.c_void_p()
    _check(lib().bcv_plan_interactions(tree.handle, ctypes.byref(opts), device, ctypes.byref(h)))
    return Plan(h, device)


def _dev_ptr(t, n, device, name):
    import torch

    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("%s must be a contiguous float64 CUDA tensor" % name)
    if t.numel() != n or t.device.index != device:
        raise ValueError("%s must hold %d values on cuda:%d" % (name, n, device))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream, device):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def vtv_apply(plan, f, u, stream=None):
    """u <- VtV potential of density f (device tensors of plan.n_dofs values: leaf order, or the
    basis layout of basis_degree=1 plans); stream-ordered."""
    n = plan.n_dofs
    _check(lib().bcv_vtv_apply(plan.handle, _dev_ptr(f, n, plan.device, "f"), _dev_ptr(u, n, plan.device, "u"),
                               _stream(stream, plan.device)))


def vtv_apply_batched(plans, fs, us, stream=None):
    """u_i <- VtV potential of f_i for every plan i, one after another on one stream
    (bcv_vtv_apply_batched); fs, us: float64 device tensors, one per plan."""
    n = len(plans)
    if not (len(fs) == n and len(us) == n and n > 0):
        raise ValueError("one density and one potential per plan")
    dev = plans[0].device
    hp = (ctypes.c_void_p * n)(*[p.handle for p in plans])
    fp = (ctypes.c_void_p * n)(*[_dev_ptr(f, p.n_dofs, p.device, "f") for p, f in zip(plans, fs)])
    up = (ctypes.c_void_p * n)(*[_dev_ptr(u, p.n_dofs, p.device, "u") for p, u in zip(plans, us)])
    _check(lib().bcv_vtv_apply_batched(hp, n, fp, up, _stream(stream, dev)))


def vtv_apply_parts(plan, f, u, parts, stream=None):
    n = plan.n_dofs
    _check(lib().bcv_vtv_apply_parts(plan.handle, _dev_ptr(f, n, plan.device, "f"),
                                     _dev_ptr(u, n, plan.device, "u"), _stream(stream, plan.device), parts))


def vtb_apply(plan, f, u_face, stream=None):
    """u_face = <1_f, N f> on every boundary face (Algorithm 2); f per leaf, u_face per face in
    Tree.faces() order (float64 device tensors; u_face overwritten)."""
    _check(lib().bcv_vtb_apply(plan.handle, _dev_ptr(f, plan.n_leaves, plan.device, "f"),
                               _dev_ptr(u_face, plan.info["n_faces"], plan.device, "u_face"),
                               _stream(stream, plan.device)))


def btv_apply(plan, q_face, g_face, u, stream=None):
    """u = <1_w, V[q] - K[g]> on every leaf (Algorithm 3); q_face, g_face per boundary face in
    Tree.faces() order (float64 device tensors), u per leaf (overwritten)."""
    nf, n = plan.info["n_faces"], plan.n_leaves
    _check(lib().bcv_btv_apply(plan.handle, _dev_ptr(q_face, nf, plan.device, "q_face"),
                               _dev_ptr(g_face, nf, plan.device, "g_face"), _dev_ptr(u, n, plan.device, "u"),
                               _stream(stream, plan.device)))


def boundary_touching_integrals():
    """(V, K): the library's 162-class tables of touching (cell, boundary face) integrals (bcv.h)."""
    V = np.empty(162)
    K = np.empty(162)
    _check(lib().bcv_boundary_touching_integrals(_dp(V), _dp(K)))
    return V, K


PHASES = ("p2m", "m2m", "m2l", "l2l", "near", "eval")


def plan_enable_timing(plan, max_applies):
    _check(lib().bcv_plan_enable_timing(plan.handle, max_applies))


def plan_phase_times(plan):
    """(total ms per phase as a dict, number of recorded applies)."""
    ms = (ctypes.c_double * len(PHASES))()
    n = ctypes.c_int64()
    _check(lib().bcv_plan_phase_times(plan.handle, ms, ctypes.byref(n)))
    return dict(zip(PHASES, list(ms))), n.value


def touching_integrals(device=0):
    out = np.empty(7)
    _check(lib().bcv_touching_integrals(device, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def n_basis(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def touching_basis_block(p_t, p_s, side_t, side_s, offset):
    """Exact touching block of the degree-p leaf bases (unit scale, without 1/(4 pi)): an array
    (n_basis(p_t), n_basis(p_s)); see bcv_touching_basis_block."""
    out = np.empty((n_basis(p_t), n_basis(p_s)))
    off = (ctypes.c_int * 3)(*[int(v) for v in offset])
    _check(lib().bcv_touching_basis_block(p_t, p_s, side_t, side_s, off,
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


# ---- touching-pair surrogate ---------------------------------------------------------------------

def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def box_pair_integrals(geom, n_gauss=16, device=0):
    """int_A int_B 1/|x-y| for boxes given as rows (A lo, A hi, B lo, B hi) of 12 doubles."""
    geom = np.ascontiguousarray(geom, dtype=np.float64).reshape(-1, 12)
    out = np.empty(len(geom))
    _check(lib().bcv_box_pair_integrals(device, len(geom), _dp(geom), n_gauss, _dp(out)))
    return out


def touch_pairs(contact, rho, off0=0.0, off1=0.0):
    """Array of canonical touching pairs from broadcast arrays of parameters."""
    contact, rho, off0, off1 = np.broadcast_arrays(np.asarray(contact), np.asarray(rho, dtype=np.float64),
                                                   np.asarray(off0, dtype=np.float64),
                                                   np.asarray(off1, dtype=np.float64))
    arr = (TouchPair * contact.size)()
    for i, (c, r, a, b) in enumerate(zip(contact.ravel(), rho.ravel(), off0.ravel(), off1.ravel())):
        arr[i].contact, arr[i].rho = int(c), float(r)
        arr[i].off[0], arr[i].off[1] = float(a), float(b)
    return arr


def touch_pair_quadrature(pairs, n_gauss=16, device=0):
    out = np.empty(len(pairs))
    _check(lib().bcv_touch_pair_quadrature(device, len(pairs), pairs, n_gauss, _dp(out)))
    return out


class MLP:
    def __init__(self, handle, device):
        self._h = handle
        self.device = device

    @property
    def handle(self):
        return self._h

    def num_params(self):
        n = ctypes.c_int64()
        _check(lib().bcv_mlp_num_params(self._h, ctypes.byref(n)))
        return n.value

    def get_params(self):
        p = np.empty(self.num_params(), dtype=np.float32)
        _check(lib().bcv_mlp_get_params(self._h, _fp(p)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.num_params()
        _check(lib().bcv_mlp_set_params(self._h, _fp(p)))

    def forward(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, 6)
        Y = np.empty((len(X), 2), dtype=np.float32)
        _check(lib().bcv_mlp_forward(self._h, len(X), _fp(X), _fp(Y)))
        return Y

    def forward_noalloc(self, X, Y, stream=None):
        """Y <- network(X) on device tensors (X: contiguous float32 CUDA [n, 6], Y: [n, 2]) with the
        library's fixed workspace: no allocation, stream-ordered (bcv_mlp_forward_noalloc)."""
        import torch

        for name, t, cols in (("X", X, 6), ("Y", Y, 2)):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
                    and t.dim() == 2 and t.shape[1] == cols and t.device.index == self.device):
                raise ValueError("%s must be a contiguous float32 CUDA tensor [n, %d] on cuda:%d"
                                 % (name, cols, self.device))
        if X.shape[0] != Y.shape[0]:
            raise ValueError("X and Y must have the same number of rows")
        _check(lib().bcv_mlp_forward_noalloc(self._h, X.shape[0], ctypes.c_void_p(X.data_ptr()),
                                             ctypes.c_void_p(Y.data_ptr()), _stream(stream, self.device)))

    def loss_grad(self, X, r):
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, 6)
        r = np.ascontiguousarray(r, dtype=np.float32)
        g = np.empty(self.num_params(), dtype=np.float32)
        loss = ctypes.c_double()
        _check(lib().bcv_mlp_loss_grad(self._h, len(X), _fp(X), _fp(r), ctypes.byref(loss), _fp(g)))
        return loss.value, g

    def train(self, n_train=100000, n_valid=4000, epochs=40, batch=1024, lr=2e-3, seed=42, n_gauss_lo=4,
              n_gauss_hi=16, tol=1e-7):
        opts = TrainOpts(n_train, n_valid, epochs, batch, lr, seed, n_gauss_lo, n_gauss_hi, tol)
        rep = TrainReport()
        _check(lib().bcv_mlp_train(self._h, ctypes.byref(opts), ctypes.byref(rep)))
        return {n: getattr(rep, n) for n, _ in TrainReport._fields_}

    def eval(self, pairs, tol=1e-7):
        n = len(pairs)
        value, est = np.empty(n), np.empty(n)
        fb = np.empty(n, dtype=np.int32)
        nf = ctypes.c_int64()
        _check(lib().bcv_surrogate_eval(self._h, n, pairs, tol, _dp(value), _dp(est),
                                        fb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(nf)))
        return value, est, fb.astype(bool)

    def save(self, path):
        _check(lib().bcv_mlp_save(self._h, os.fsencode(path)))

    def destroy(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.bcv_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        self.destroy()


def mlp_create(width=128, seed=0, device=0):
    h = ctypes.c_void_p()
    _check(lib().bcv_mlp_create(width, seed, device, ctypes.byref(h)))
    return MLP(h, device)


def mapped_pair_entries(geom_t, geom_s, device=0):
    """Entries of touching pairs of cube-to-ball mapped cells by the planner's singular rule (rows: lower
    corner in the reference cube [0,1]^3 and side of each cube)."""
    gt = np.ascontiguousarray(geom_t, dtype=np.float64).reshape(-1, 4)
    gs = np.ascontiguousarray(geom_s, dtype=np.float64).reshape(-1, 4)
    if len(gt) != len(gs):
        raise ValueError("one partner per cube")
    value = np.empty(len(gt))
    _check(lib().bcv_mapped_pair_entries(device, len(gt), _dp(gt), _dp(gs), _dp(value)))
    return value


def mlp_load(path, device=0):
    h = ctypes.c_void_p()
    _check(lib().bcv_mlp_load(os.fsencode(path), device, ctypes.byref(h)))
    return MLP(h, device)


# ---- captured applies and the autotuner ------------------------------------------------------------

class Graph:
    """bcv_vtv_apply captured into one HIP graph; keeps f and u (torch tensors) alive."""

    def __init__(self, handle, plan, f, u):
        self._h, self._plan, self.f, self.u = handle, plan, f, u

    def launch(self, stream=None):
        _check(lib().bcv_graph_launch(self._h, _stream(stream, self._plan.device)))

    def destroy(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.bcv_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        self.destroy()


def vtv_graph_create(plan, f, u):
    n = plan.n_dofs
    h = ctypes.c_void_p()
    _check(lib().bcv_vtv_graph_create(plan.handle, _dev_ptr(f, n, plan.device, "f"), _dev_ptr(u, n, plan.device, "u"),
                                      ctypes.byref(h)))
    return Graph(h, plan, f, u)


def autotune(tree, device=0, n_applies=5, **opts):
    """Best (near_unit, m2l_max_slots) for the tree and options, and its ms per apply."""
    base = _opts(**opts)
    best = PlanOpts()
    ms = ctypes.c_double()
    _check(lib().bcv_autotune(tree.handle, ctypes.byref(base), device, n_applies, ctypes.byref(best), ctypes.byref(ms)))
    return {"near_unit": best.near_unit, "m2l_max_slots": best.m2l_max_slots}, ms.value
