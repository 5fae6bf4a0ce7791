"""ctypes binding of libadjoint.so (include/adjoint.h).

Argument marshalling only: the functions below take torch tensors (device
memory) or NumPy arrays (host memory), pass raw pointers and sizes to the C
ABI and raise on a non-zero status.  Every step of the adjoint runs in the
HIP kernels of the library.  Loading fails loudly when the library has not
been built; there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadjoint.so")

STATUS = {0: "ADJ_OK", -1: "ADJ_E_ARG", -2: "ADJ_E_SHAPE", -3: "ADJ_E_INVERTED",
          -4: "ADJ_E_NOCONV", -5: "ADJ_E_SINGULAR", -6: "ADJ_E_DEVICE", -7: "ADJ_E_OOM",
          -8: "ADJ_E_NOTIMPL"}
ADJ_FP64, ADJ_MIXED, ADJ_MIXED_PC = 0, 1, 2
ADJ_AUTO, ADJ_GMRES, ADJ_PCG, ADJ_SEMI_IMPLICIT = 0, 1, 2, 3
PRECOND_WOODBURY, PRECOND_SPARSE_INVERSE, PRECOND_JACOBI, PRECOND_POINT_JACOBI = 0, 1, 2, 3
PRECOND_WOODBURY_NO_Z = 4
MAT_NEO_HOOKEAN, MAT_ARAP, MAT_COROT = 0, 1, 2
MATERIAL_CODES = {"nh": MAT_NEO_HOOKEAN, "arap": MAT_ARAP, "corot": MAT_COROT}

# names declared in include/adjoint.h
EXPORTS = ("adj_scene_create", "adj_scene_destroy", "adjoint_setup", "adjoint_solve", "vjp_params",
           "vjp_params_noalloc", "sim_forward_step", "adj_scene_info", "adj_check_status", "adj_debug_export",
           "adj_profile_begin", "adj_profile_end", "adj_forward_stats", "adj_forward_reset", "adj_set_spheres",
           "adj_set_binding_targets",
           "adj_set_actuation", "adj_actuation_force", "adj_actuation_vjp",
           "adj_set_tuning", "adj_get_tuning", "adj_autotune", "adj_batch_create", "adj_batch_destroy",
           "adj_batch_info", "adj_batch_setup", "adj_batch_solve", "adj_batch_vjp", "adj_batch_check_status",
           "adj_batch_debug_export", "adj_batch_scene", "adj_batch_reverse", "adj_binding_vjp",
           "adj_batch_set_tuning", "adj_batch_get_tuning", "adj_batch_autotune", "adj_last_error")
KERNELS = {"S": 0, "ST": 1, "capinv": 2, "Z": 3, "correction": 3, "bsr": 4, "tet": 5, "assemble": 6, "gj": 7,
           "gs_pass2": 8, "gs_pass1": 9, "gj_step": 10, "delassus": 11, "lu_tiles": 12}


class AdjError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class SceneDesc(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tets", C.c_int32), ("rest_pos", C.c_void_p),
                ("tets", C.c_void_p), ("density", C.c_double), ("h", C.c_double), ("eps", C.c_double),
                ("E", C.c_void_p), ("nu", C.c_void_p), ("per_tet_material", C.c_int32),
                ("gravity", C.c_double * 3), ("n_planes", C.c_int32), ("planes", C.c_void_p),
                ("contact_margin", C.c_double), ("n_bindings", C.c_int32), ("binding_vid", C.c_void_p),
                ("binding_E", C.c_void_p), ("material", C.c_int32)]


class ContactState(C.Structure):
    _fields_ = [("n_contacts", C.c_int32), ("capacity", C.c_int32), ("vid", C.c_void_p),
                ("fric", C.c_void_p), ("frame", C.c_void_p), ("delta", C.c_void_p),
                ("lam", C.c_void_p), ("d_n", C.c_void_p), ("d_f", C.c_void_p), ("mu", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32), ("restart", C.c_int32),
                ("max_refine", C.c_int32), ("prec", C.c_int32), ("reuse_delassus", C.c_int32),
                ("method", C.c_int32), ("precond", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("refine_steps", C.c_int32), ("n_contacts", C.c_int32),
                ("m_rows", C.c_int32), ("relres", C.c_double), ("delassus_rebuilt", C.c_int32),
                ("method", C.c_int32)]


class BatchTuning(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("graph", C.c_int32), ("a_inv", C.c_int32)]

    def as_dict(self):
        return {"chunk": self.chunk, "graph": self.graph, "a_inv": self.a_inv}


class Tuning(C.Structure):
    _fields_ = [("gs_rows", C.c_int32), ("bsr_lanes", C.c_int32), ("chunk", C.c_int32), ("graph", C.c_int32),
                ("gj_wide_min", C.c_int32), ("a_inv", C.c_int32), ("lu_min", C.c_int32), ("lu_pipe", C.c_int32),
                ("sweep_fuse", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2603_16478_amd.build.build() first")
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.adj_last_error.restype = C.c_char_p
    lib.adj_scene_create.argtypes = [C.POINTER(SceneDesc), C.c_int32, C.POINTER(vp)]
    lib.adj_scene_destroy.argtypes = [vp]
    lib.adjoint_setup.argtypes = [vp, C.POINTER(ContactState), vp, C.POINTER(SolveOpts), vp]
    lib.adjoint_solve.argtypes = [vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
    lib.vjp_params.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.vjp_params_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.sim_forward_step.argtypes = [vp, vp, vp, vp, C.c_double, vp, vp, C.POINTER(ContactState), vp]
    lib.adj_scene_info.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.adj_check_status.argtypes = [vp, vp]
    lib.adj_debug_export.argtypes = [vp, C.c_int32, vp, C.c_int64, C.POINTER(C.c_int64)]
    lib.adj_profile_begin.argtypes = [vp, C.c_int32]
    lib.adj_forward_stats.argtypes = [vp, C.POINTER(C.c_double)]
    lib.adj_forward_reset.argtypes = [vp]
    lib.adj_set_spheres.argtypes = [vp, C.c_int32, vp, vp]
    lib.adj_set_binding_targets.argtypes = [vp, vp]
    lib.adj_set_actuation.argtypes = [vp, C.c_int32, vp, vp]
    lib.adj_actuation_force.argtypes = [vp, vp, vp, vp]
    lib.adj_actuation_vjp.argtypes = [vp, vp, vp, vp]
    lib.adj_profile_end.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.adj_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
    lib.adj_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
    lib.adj_autotune.argtypes = [vp, vp, vp, vp, C.POINTER(SolveOpts), C.c_int32, C.POINTER(Tuning), vp]
    lib.adj_batch_set_tuning.argtypes = [vp, C.POINTER(BatchTuning)]
    lib.adj_batch_get_tuning.argtypes = [vp, C.POINTER(BatchTuning)]
    lib.adj_batch_autotune.argtypes = [vp, vp, vp, vp, C.POINTER(SolveOpts), C.c_int32, C.POINTER(BatchTuning), vp]
    lib.adj_batch_create.argtypes = [C.c_int32, C.POINTER(SceneDesc), C.POINTER(C.c_int32), C.POINTER(vp)]
    lib.adj_batch_destroy.argtypes = [vp]
    lib.adj_batch_info.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.adj_batch_setup.argtypes = [vp, C.POINTER(ContactState), vp, C.POINTER(SolveOpts), vp]
    lib.adj_batch_solve.argtypes = [vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
    lib.adj_batch_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.adj_batch_check_status.argtypes = [vp, vp]
    lib.adj_batch_debug_export.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_int64, C.POINTER(C.c_int64)]
    lib.adj_batch_scene.argtypes = [vp, C.POINTER(vp)]
    lib.adj_binding_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.adj_batch_reverse.argtypes = [vp, vp, C.c_int32, C.POINTER(ContactState), C.POINTER(vp), vp, vp,
                                      C.POINTER(vp), vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
    for name in EXPORTS:
        if name != "adj_last_error":
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def check(status: int):
    if status != 0:
        raise AdjError(status, load().adj_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream


class Scene:
    """Owns an adj_scene (adj_scene_create / adj_scene_destroy)."""

    def __init__(self, rest, tets, density, h, eps, E, nu, gravity, planes, contact_margin,
                 max_contacts, bindings=None, material=0):
        """bindings: None or (vertex ids, compliances) of bilateral bindings;
        material: MAT_NEO_HOOKEAN, MAT_ARAP or MAT_COROT."""
        lib = load()
        self._keep = []
        rest = np.ascontiguousarray(rest, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        E = np.ascontiguousarray(np.atleast_1d(E), dtype=np.float64)
        nu = np.ascontiguousarray(np.atleast_1d(nu), dtype=np.float64)
        planes = np.ascontiguousarray(np.asarray(planes, dtype=np.float64).reshape(-1, 4))
        self._keep += [rest, tets, E, nu, planes]
        d = SceneDesc()
        d.n_verts, d.n_tets = rest.shape[0], tets.shape[0]
        d.rest_pos, d.tets = rest.ctypes.data, tets.ctypes.data
        d.density, d.h, d.eps = float(density), float(h), float(eps)
        d.E, d.nu = E.ctypes.data, nu.ctypes.data
        d.per_tet_material = 1 if E.shape[0] == tets.shape[0] and tets.shape[0] > 1 else 0
        d.gravity = (C.c_double * 3)(*[float(g) for g in gravity])
        d.n_planes = planes.shape[0]
        d.planes = planes.ctypes.data if planes.shape[0] else None
        d.contact_margin = float(contact_margin)
        d.material = int(material)
        self.n_bindings = 0
        if bindings is not None:
            bvid = np.ascontiguousarray(bindings[0], dtype=np.int32)
            bE = np.ascontiguousarray(np.broadcast_to(np.asarray(bindings[1], dtype=np.float64), bvid.shape))
            self._keep += [bvid, bE]
            d.n_bindings = bvid.shape[0]
            d.binding_vid, d.binding_E = bvid.ctypes.data, bE.ctypes.data
            self.n_bindings = int(bvid.shape[0])
        handle = C.c_void_p()
        check(lib.adj_scene_create(C.byref(d), int(max_contacts), C.byref(handle)))
        self.handle = handle
        self.n_verts, self.n_tets, self.h = d.n_verts, d.n_tets, d.h

    def info(self):
        out = (C.c_int64 * 6)()
        check(load().adj_scene_info(self.handle, out))
        keys = ("n_verts", "n_tets", "nnz_blocks", "nnz_L", "nnz_S", "max_contacts")
        return dict(zip(keys, list(out)))

    def close(self):
        if getattr(self, "handle", None):
            check(load().adj_scene_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_contact_state(n, vid, fric, frame, delta, lam, mu, d_n=None, d_f=None, capacity=None):
    """Fill an adj_contact_state from device tensors (sorted by vertex)."""
    cs = ContactState()
    cs.n_contacts = int(n)
    cs.capacity = int(capacity if capacity is not None else n)
    cs.vid, cs.fric, cs.frame = _ptr(vid), _ptr(fric), _ptr(frame)
    cs.delta, cs.lam = _ptr(delta), _ptr(lam)
    cs.d_n, cs.d_f = _ptr(d_n), _ptr(d_f)
    cs.mu = float(mu)
    return cs


def solve_opts(rtol=1e-8, maxit=2000, restart=64, prec=ADJ_FP64, reuse_delassus=1, max_refine=4,
               method=ADJ_AUTO, precond=0):
    o = SolveOpts()
    o.rtol, o.maxit, o.restart, o.max_refine = float(rtol), int(maxit), int(restart), int(max_refine)
    o.prec, o.reuse_delassus, o.method, o.precond = int(prec), int(reuse_delassus), int(method), int(precond)
    return o


def adjoint_setup(scene: Scene, contacts: ContactState, q, opts: SolveOpts, stream=None):
    check(load().adjoint_setup(scene.handle, C.byref(contacts), _ptr(q), C.byref(opts), _stream(stream)))


def adjoint_solve(scene: Scene, dL_dq, dL_dv, z, opts: SolveOpts, stream=None, raise_noconv=True):
    info = SolveInfo()
    st = load().adjoint_solve(scene.handle, _ptr(dL_dq), _ptr(dL_dv), _ptr(z), C.byref(opts),
                              C.byref(info), _stream(stream))
    if st != 0 and not (st == -4 and not raise_noconv):
        check(st)
    return info


def vjp_params(scene: Scene, z, dL_dv, dL_dqbar, dL_dvbar, dL_dfext, grad3, dE_tet=None, dnu_tet=None,
               stream=None):
    check(load().vjp_params(scene.handle, _ptr(z), _ptr(dL_dv), _ptr(dL_dqbar), _ptr(dL_dvbar),
                            _ptr(dL_dfext), _ptr(grad3), _ptr(dE_tet), _ptr(dnu_tet), _stream(stream)))


def vjp_params_noalloc(scene: Scene, z, dL_dv, dL_dqbar, dL_dvbar, dL_dfext, grad3, dE_tet=None, dnu_tet=None,
                       stream=None):
    """vjp_params without any device allocation (fixed library scratch)."""
    check(load().vjp_params_noalloc(scene.handle, _ptr(z), _ptr(dL_dv), _ptr(dL_dqbar), _ptr(dL_dvbar),
                                    _ptr(dL_dfext), _ptr(grad3), _ptr(dE_tet), _ptr(dnu_tet), _stream(stream)))


_DEBUG = {0: ("val", np.float64), 1: ("rowptr", np.int32), 2: ("col", np.int32),
          3: ("capinv", np.float64), 4: ("delassus", np.float64), 5: ("Q", np.float64),
          6: ("lu_pivots", np.float64)}


def debug_export(scene: Scene, what: int) -> np.ndarray:
    lib = load()
    size = C.c_int64()
    lib.adj_debug_export(scene.handle, int(what), None, 0, C.byref(size))
    out = np.empty(max(size.value, 1) // np.dtype(_DEBUG[what][1]).itemsize, dtype=_DEBUG[what][1])
    check(lib.adj_debug_export(scene.handle, int(what), out.ctypes.data, out.nbytes, C.byref(size)))
    return out[: size.value // out.itemsize]


def profile_begin(scene: Scene, kernel: str):
    check(load().adj_profile_begin(scene.handle, KERNELS[kernel]))


def profile_end(scene: Scene):
    ms, n = C.c_double(), C.c_int64()
    check(load().adj_profile_end(scene.handle, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def binding_vjp(scene: Scene, z, q, targets, dL_dtargets, dL_dE, stream=None):
    """dL/dd_b and dL/dE_b of the bilateral bindings (adj_binding_vjp)."""
    check(load().adj_binding_vjp(scene.handle, _ptr(z), _ptr(q), _ptr(targets), _ptr(dL_dtargets), _ptr(dL_dE),
                                 _stream(stream)))


def check_status(scene: Scene, stream=None):
    check(load().adj_check_status(scene.handle, _stream(stream)))


def sim_forward_step(scene: Scene, qbar, vbar, f_ext, mu, q, v, contacts: ContactState, stream=None):
    check(load().sim_forward_step(scene.handle, _ptr(qbar), _ptr(vbar), _ptr(f_ext), float(mu), _ptr(q),
                                  _ptr(v), C.byref(contacts), _stream(stream)))


def forward_stats(scene: Scene):
    out = (C.c_double * 2)()
    check(load().adj_forward_stats(scene.handle, out))
    return int(out[0]), float(out[1])


def forward_reset(scene: Scene):
    check(load().adj_forward_reset(scene.handle))


def set_actuation(scene: Scene, group, fibre, n_groups):
    """Actuation groups (0 .. n_groups-1) and fibre directions per tet
    (adj_set_actuation)."""
    g = np.ascontiguousarray(group, dtype=np.int32)
    d = np.ascontiguousarray(np.asarray(fibre, dtype=np.float64).reshape(-1, 3))
    if g.shape[0] != scene.n_tets or d.shape[0] != scene.n_tets:
        raise ValueError("one group and one fibre per tet")
    check(load().adj_set_actuation(scene.handle, int(n_groups), g.ctypes.data, d.ctypes.data))


def actuation_force(scene: Scene, a, f, stream=None):
    """f = Phi a (adj_actuation_force)."""
    check(load().adj_actuation_force(scene.handle, _ptr(a), _ptr(f), _stream(stream)))


def actuation_vjp(scene: Scene, dL_df, dL_da, stream=None):
    """dL/da = Phi^T dL/df (adj_actuation_vjp)."""
    check(load().adj_actuation_vjp(scene.handle, _ptr(dL_df), _ptr(dL_da), _stream(stream)))


def set_binding_targets(scene: Scene, targets):
    """Binding targets d_b of the next forward steps (adj_set_binding_targets);
    targets (n_b, 3) host array in the order of the scene's bindings."""
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.float64).reshape(-1))
    check(load().adj_set_binding_targets(scene.handle, t.ctypes.data))


def set_spheres(scene: Scene, old_pose, new_pose):
    """Kinematic spheres of the next forward steps (adj_set_spheres); poses
    (n, 4) host arrays of (centre, radius)."""
    old = np.ascontiguousarray(np.asarray(old_pose, dtype=np.float64).reshape(-1, 4))
    new = np.ascontiguousarray(np.asarray(new_pose, dtype=np.float64).reshape(-1, 4))
    if old.shape != new.shape:
        raise ValueError("old and new sphere poses differ in shape")
    n = old.shape[0]
    check(load().adj_set_spheres(scene.handle, n, old.ctypes.data if n else None, new.ctypes.data if n else None))


class ContactBuffers:
    """Device arrays for one step record (capacity entries) and the
    adj_contact_state that points at them."""

    def __init__(self, capacity, device="cuda"):
        import torch
        n = max(int(capacity), 1)
        self.vid = torch.zeros(n, dtype=torch.int32, device=device)
        self.fric = torch.zeros(n, dtype=torch.int32, device=device)
        self.frame = torch.zeros(n, 9, dtype=torch.float64, device=device)
        self.delta = torch.zeros(n, 3, dtype=torch.float64, device=device)
        self.lam = torch.zeros(n, 3, dtype=torch.float64, device=device)
        self.d_n = torch.zeros(n, dtype=torch.float64, device=device)
        self.d_f = torch.zeros(n, 2, dtype=torch.float64, device=device)
        self.state = make_contact_state(0, self.vid, self.fric, self.frame, self.delta, self.lam, 0.0,
                                        self.d_n, self.d_f, capacity=capacity)

    @property
    def n(self):
        return int(self.state.n_contacts)

    def clone(self):
        """A copy of the current record (device tensors) with its own state."""
        c = ContactBuffers.__new__(ContactBuffers)
        for k in ("vid", "fric", "frame", "delta", "lam", "d_n", "d_f"):
            setattr(c, k, getattr(self, k).clone())
        c.state = make_contact_state(self.state.n_contacts, c.vid, c.fric, c.frame, c.delta, c.lam,
                                     self.state.mu, c.d_n, c.d_f, capacity=self.state.capacity)
        return c


def set_tuning(scene: Scene, gs_rows=64, bsr_lanes=16, chunk=8, graph=0, gj_wide_min=2048, a_inv=0, lu_min=4608,
               lu_pipe=1, sweep_fuse=0):
    t = Tuning(int(gs_rows), int(bsr_lanes), int(chunk), int(graph), int(gj_wide_min), int(a_inv), int(lu_min),
               int(lu_pipe), int(sweep_fuse))
    check(load().adj_set_tuning(scene.handle, C.byref(t)))


def get_tuning(scene: Scene) -> dict:
    t = Tuning()
    check(load().adj_get_tuning(scene.handle, C.byref(t)))
    return t.as_dict()


def autotune(scene: Scene, dL_dq, dL_dv, z, opts: SolveOpts, reps=3, stream=None) -> dict:
    """Time candidate launch shapes on the set-up scene and keep the fastest."""
    t = Tuning()
    check(load().adj_autotune(scene.handle, _ptr(dL_dq), _ptr(dL_dv), _ptr(z), C.byref(opts), int(reps),
                              C.byref(t), _stream(stream)))
    return t.as_dict()


class _SceneRef:
    """Non-owning reference to a scene handle."""

    def __init__(self, handle):
        self.handle = handle

    def info(self):
        out = (C.c_int64 * 6)()
        check(load().adj_scene_info(self.handle, out))
        keys = ("n_verts", "n_tets", "nnz_blocks", "nnz_L", "nnz_S", "max_contacts")
        return dict(zip(keys, list(out)))


class Batch:
    """Owns an adj_batch: several scenes solved together (adj_batch_create).
    specs: sequence of (rest, tets, E, nu); density, h, eps are shared."""

    def __init__(self, specs, density, h, eps, gravity, planes, contact_margin, max_contacts, bindings=None,
                 material=0):
        """bindings: None, or per scene None / (vertex ids, compliances);
        material: the scenes' common material model."""
        lib = load()
        self._keep = []
        n = len(specs)
        descs = (SceneDesc * n)()
        planes = np.ascontiguousarray(np.asarray(planes, dtype=np.float64).reshape(-1, 4))
        self._keep.append(planes)
        for k, (rest, tets, E, nu) in enumerate(specs):
            rest = np.ascontiguousarray(rest, dtype=np.float64)
            tets = np.ascontiguousarray(tets, dtype=np.int32)
            E = np.ascontiguousarray(np.atleast_1d(E), dtype=np.float64)
            nu = np.ascontiguousarray(np.atleast_1d(nu), dtype=np.float64)
            self._keep += [rest, tets, E, nu]
            d = descs[k]
            d.n_verts, d.n_tets = rest.shape[0], tets.shape[0]
            d.rest_pos, d.tets = rest.ctypes.data, tets.ctypes.data
            d.density, d.h, d.eps = float(density), float(h), float(eps)
            d.E, d.nu = E.ctypes.data, nu.ctypes.data
            d.per_tet_material = 1 if E.shape[0] == tets.shape[0] and tets.shape[0] > 1 else 0
            d.gravity = (C.c_double * 3)(*[float(g) for g in gravity])
            d.n_planes = planes.shape[0]
            d.planes = planes.ctypes.data if planes.shape[0] else None
            d.contact_margin = float(contact_margin)
            d.material = int(material)
            if bindings is not None and bindings[k] is not None:
                bvid = np.ascontiguousarray(bindings[k][0], dtype=np.int32)
                bE = np.ascontiguousarray(np.broadcast_to(np.asarray(bindings[k][1], dtype=np.float64), bvid.shape))
                self._keep += [bvid, bE]
                d.n_bindings = bvid.shape[0]
                d.binding_vid, d.binding_E = bvid.ctypes.data, bE.ctypes.data
        mc = (C.c_int32 * n)(*[int(m) for m in max_contacts])
        handle = C.c_void_p()
        check(lib.adj_batch_create(n, descs, mc, C.byref(handle)))
        self.handle, self.n_scenes = handle, n
        out = (C.c_int64 * (2 * (n + 1)))()
        check(lib.adj_batch_info(handle, out))
        self.voff = np.array(list(out)[: n + 1], dtype=np.int64)
        self.toff = np.array(list(out)[n + 1:], dtype=np.int64)

    def union_scene(self):
        """The batch's union scene (for profile_begin/end and info); owned by the batch."""
        h = C.c_void_p()
        check(load().adj_batch_scene(self.handle, C.byref(h)))
        return _SceneRef(h)

    def close(self):
        if getattr(self, "handle", None):
            check(load().adj_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_setup(batch: Batch, contacts, q, opts: SolveOpts, stream=None):
    """contacts: list of ContactState (one per scene); q: packed device tensor."""
    arr = (ContactState * batch.n_scenes)(*contacts)
    check(load().adj_batch_setup(batch.handle, arr, _ptr(q), C.byref(opts), _stream(stream)))


def batch_solve(batch: Batch, dL_dq, dL_dv, z, opts: SolveOpts, stream=None, raise_noconv=True):
    infos = (SolveInfo * batch.n_scenes)()
    st = load().adj_batch_solve(batch.handle, _ptr(dL_dq), _ptr(dL_dv), _ptr(z), C.byref(opts), infos,
                                _stream(stream))
    if st != 0 and (raise_noconv or STATUS.get(st) != "ADJ_E_NOCONV"):
        check(st)
    return list(infos)


def batch_vjp(batch: Batch, z, dL_dv, dL_dqbar, dL_dvbar, dL_dfext, grad, stream=None):
    check(load().adj_batch_vjp(batch.handle, _ptr(z), _ptr(dL_dv), _ptr(dL_dqbar), _ptr(dL_dvbar),
                               _ptr(dL_dfext), _ptr(grad), _stream(stream)))


def batch_reverse(b0: Batch, b1: Batch, contacts, q, gq, gv, dfext, grad, opts: SolveOpts, stream=None,
                  raise_noconv=True):
    """Reverse pass over len(q) recorded steps (adj_batch_reverse): contacts[t]
    is the list of per-scene ContactState of step t, q[t] its packed state;
    gq, gv are updated in place; dfext: list of packed outputs or None.
    Returns the per-step lists of SolveInfo."""
    T, ns = len(q), b0.n_scenes
    flat = [c for step in contacts for c in step]
    if len(contacts) != T or len(flat) != T * ns:
        raise ValueError("contacts must hold n_scenes states for every step")
    carr = (ContactState * (T * ns))(*flat)
    qarr = (C.c_void_p * T)(*[_ptr(x) for x in q])
    darr = None if dfext is None else (C.c_void_p * T)(*[_ptr(x) for x in dfext])
    infos = (SolveInfo * (T * ns))()
    st = load().adj_batch_reverse(b0.handle, b1.handle, int(T), carr, qarr, _ptr(gq), _ptr(gv), darr, _ptr(grad),
                                  C.byref(opts), infos, _stream(stream))
    if st != 0 and (raise_noconv or STATUS.get(st) != "ADJ_E_NOCONV"):
        check(st)
    return [list(infos[t * ns:(t + 1) * ns]) for t in range(T)]


def batch_set_tuning(batch: Batch, chunk=8, graph=0, a_inv=0):
    t = BatchTuning(int(chunk), int(graph), int(a_inv))
    check(load().adj_batch_set_tuning(batch.handle, C.byref(t)))


def batch_get_tuning(batch: Batch) -> dict:
    t = BatchTuning()
    check(load().adj_batch_get_tuning(batch.handle, C.byref(t)))
    return t.as_dict()


def batch_autotune(batch: Batch, dL_dq, dL_dv, z, opts: SolveOpts, reps=2, stream=None) -> dict:
    """Time A^-1 by products or sweeps, chunk sizes and graph replay on the set-up batch; keep the fastest."""
    t = BatchTuning()
    check(load().adj_batch_autotune(batch.handle, _ptr(dL_dq), _ptr(dL_dv), _ptr(z), C.byref(opts), int(reps),
                                    C.byref(t), _stream(stream)))
    return t.as_dict()


def batch_check_status(batch: Batch, stream=None):
    check(load().adj_batch_check_status(batch.handle, _stream(stream)))


def batch_debug_export(batch: Batch, what: int, scene: int) -> np.ndarray:
    lib = load()
    size = C.c_int64()
    lib.adj_batch_debug_export(batch.handle, int(what), int(scene), None, 0, C.byref(size))
    out = np.empty(max(size.value, 8) // 8, dtype=np.float64)
    check(lib.adj_batch_debug_export(batch.handle, int(what), int(scene), out.ctypes.data, out.nbytes,
                                     C.byref(size)))
    return out[: size.value // 8]
