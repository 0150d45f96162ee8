"""Thin Python binding of libhofv: argument marshalling only.

Device vectors are torch tensors on the HIP device, float64, laid out
component-major ([dim][n_cells], i.e. shape (dim, n_cells), contiguous).  Every
computation happens in the library; this module only passes pointers, sizes
and options, and evaluates the caller's boundary/body-force functions at the
points the library reports (those functions are problem inputs).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


class HofvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{L.STATUS.get(status, status)}: {msg}")
        self.status = status


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 HIP tensor")
    if numel is not None and t.numel() != numel:  # the kernels index by the mesh's size
        raise ValueError(f"expected a tensor of {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


class Context:
    """One discretisation on one device (hofv_ctx)."""

    def __init__(self, dim, order_p, n_plus, n_gauss, material, mu, lam, alpha=0.1, k_weight=6.0,
                 ghost_weight=1.0, stencil_quantum=1e-12, fold_quadrature=True, host_only=False, precond_levels=1,
                 face_rule=0, stencil_grow=0):
        self.lib = L.load()
        prm = L.Params(dim, order_p, n_plus, n_gauss, material, int(bool(fold_quadrature)), mu, lam, alpha,
                       k_weight, ghost_weight, stencil_quantum, int(bool(host_only)), int(precond_levels),
                       int(face_rule), int(stencil_grow))
        h = C.c_void_p()
        st = self.lib.hofv_create(C.byref(prm), C.byref(h))
        if st != L.HOFV_OK:
            raise HofvError(st, self.lib.hofv_last_error(None).decode())
        self.h = h
        self.dim = dim
        self.params = prm
        self.n_cells = 0
        self.report = None

    def _check(self, st):
        if st != L.HOFV_OK:
            raise HofvError(st, self.lib.hofv_last_error(self.h).decode())

    def _v(self, t):
        """Pointer of a device vector [dim][n_cells] of this mesh."""
        return _ptr(t, self.dim * self.n_cells)

    def close(self):
        if getattr(self, "h", None):
            self.lib.hofv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------- setup
    def set_mesh(self, verts, cells):
        verts = np.ascontiguousarray(verts, np.float64)
        cells = np.ascontiguousarray(cells, np.int64)
        if verts.ndim != 2 or verts.shape[1] != self.dim:
            raise ValueError(f"verts must be (n_verts, {self.dim})")
        if cells.ndim != 2 or cells.shape[1] not in (2 ** self.dim, self.dim + 1):
            raise ValueError(f"cells must be (n_cells, {2 ** self.dim}) or (n_cells, {self.dim + 1})")
        # cells of dim + 1 vertices are triangles or tetrahedra
        fn = self.lib.hofv_set_mesh_simplices if cells.shape[1] == verts.shape[1] + 1 else self.lib.hofv_set_mesh
        self._check(fn(self.h, verts.shape[0], _dptr(verts), cells.shape[0],
                       cells.ctypes.data_as(C.POINTER(C.c_int64))))
        self.n_cells = cells.shape[0]

    def set_mesh_poly(self, verts, face_ptr, face_verts, face_cells, n_cells):
        """Face-list (polygonal / polyhedral) mesh: face f's vertex loop is
        face_verts[face_ptr[f]:face_ptr[f + 1]], its right-hand normal pointing
        out of face_cells[f, 0] into face_cells[f, 1] (-1: boundary)."""
        verts = np.ascontiguousarray(verts, np.float64)
        fp = np.ascontiguousarray(face_ptr, np.int64)
        fv = np.ascontiguousarray(face_verts, np.int64)
        fc = np.ascontiguousarray(face_cells, np.int64)
        if verts.ndim != 2 or verts.shape[1] != self.dim:
            raise ValueError(f"verts must be (n_verts, {self.dim})")
        nf = fc.shape[0]
        if fc.shape != (nf, 2) or fp.shape != (nf + 1,) or fv.size != fp[-1]:
            raise ValueError("face_cells must be (n_faces, 2), face_ptr (n_faces + 1,) ending at len(face_verts)")
        P64 = C.POINTER(C.c_int64)
        self._check(self.lib.hofv_set_mesh_polyhedra(self.h, verts.shape[0], _dptr(verts), int(n_cells), nf,
                                                     fp.ctypes.data_as(P64), fv.ctypes.data_as(P64),
                                                     fc.ctypes.data_as(P64)))
        self.n_cells = int(n_cells)

    def boundary_faces(self):
        n = C.c_int64()
        nq = C.c_int32()
        cen, nor, qp = (C.POINTER(C.c_double)(), C.POINTER(C.c_double)(), C.POINTER(C.c_double)())
        self._check(self.lib.hofv_boundary_faces(self.h, C.byref(n), C.byref(nq), C.byref(cen), C.byref(nor),
                                                 C.byref(qp)))
        D, nb, q = self.dim, n.value, nq.value
        as_np = lambda p, shape: np.ctypeslib.as_array(p, shape=shape).copy() if nb else np.zeros(shape)
        return as_np(cen, (nb, D)), as_np(nor, (nb, D)), as_np(qp, (nb, q, D))

    def cell_centroids(self):
        pts = C.POINTER(C.c_double)()
        self._check(self.lib.hofv_cell_centroids(self.h, C.byref(pts)))
        return np.ctypeslib.as_array(pts, shape=(self.n_cells, self.dim)).copy()

    def volume_qpoints(self):
        nqv = C.c_int32()
        pts = C.POINTER(C.c_double)()
        self._check(self.lib.hofv_volume_qpoints(self.h, C.byref(nqv), C.byref(pts)))
        return np.ctypeslib.as_array(pts, shape=(self.n_cells, nqv.value, self.dim)).copy()

    def volume_qpoints_csr(self):
        """(points (n_points, dim), cell_ptr (n_cells + 1,)): cell P's points
        are points[cell_ptr[P]:cell_ptr[P + 1]]."""
        n = C.c_int64()
        ptr = C.POINTER(C.c_int64)()
        pts = C.POINTER(C.c_double)()
        self._check(self.lib.hofv_volume_qpoints_csr(self.h, C.byref(n), C.byref(ptr), C.byref(pts)))
        cp = np.ctypeslib.as_array(ptr, shape=(self.n_cells + 1,)).copy()
        return np.ctypeslib.as_array(pts, shape=(n.value, self.dim)).copy(), cp

    def set_bc(self, types, u_b_q, u_b_centre, traction_q):
        types = np.ascontiguousarray(types, np.int32)
        arrs = [None if a is None else np.ascontiguousarray(a, np.float64) for a in (u_b_q, u_b_centre, traction_q)]
        # the library reads these sizes from the pointers: check them here
        n, nq = C.c_int64(), C.c_int32()
        self._check(self.lib.hofv_boundary_faces(self.h, C.byref(n), C.byref(nq), None, None, None))
        nb, q, D = n.value, nq.value, self.dim
        if types.shape != (nb,):
            raise ValueError(f"types must be ({nb},)")
        for a, shape in zip(arrs, ((nb, q, D), (nb, D), (nb, q, D))):
            if a is not None and a.size != nb * int(np.prod(shape[1:])):
                raise ValueError(f"boundary arrays must be {shape}")
        self._check(self.lib.hofv_set_bc(self.h, types.ctypes.data_as(C.POINTER(C.c_int32)),
                                         *[_dptr(a) for a in arrs]))

    def set_body_force(self, values):
        """f_b at every volume quadrature point, in the order of volume_qpoints_csr."""
        v = None if values is None else np.ascontiguousarray(values, np.float64)
        if v is not None:
            n = C.c_int64()
            self._check(self.lib.hofv_volume_qpoints_csr(self.h, C.byref(n), None, None))
            if v.size != n.value * self.dim:
                raise ValueError(f"body force must have {n.value} x {self.dim} values")
        self._check(self.lib.hofv_set_body_force(self.h, _dptr(v)))

    def setup(self):
        rep = L.SetupReport()
        self._check(self.lib.hofv_setup(self.h, C.byref(rep)))
        self.report = {k: getattr(rep, k) for k, _ in L.SetupReport._fields_}
        return self.report

    def set_load_scale(self, s):
        self._check(self.lib.hofv_set_load_scale(self.h, float(s)))

    def set_multigrid(self, enable):
        self._check(self.lib.hofv_set_multigrid(self.h, int(bool(enable))))

    def set_nej(self, inner_iters):
        """Near-exact Jacobian preconditioner (App. C) with inner_iters inner
        GMRES iterations per application; 0 switches it off."""
        self._check(self.lib.hofv_set_nej(self.h, int(inner_iters)))

    # ------------------------------------------------------------------- hot
    def residual(self, u, R, stream=None):
        self._check(self.lib.hofv_residual(self.h, self._v(u), self._v(R), _stream(stream)))

    def jvp(self, u, Ru, v, Jv, eps=0.0, stream=None):
        self._check(self.lib.hofv_jvp(self.h, self._v(u), self._v(Ru), self._v(v), self._v(Jv), float(eps),
                                      _stream(stream)))

    def jvp_noalloc(self, u, Ru, v, Jv, eps=0.0, stream=None):
        """jvp with its reduction scratch in the library's static device array
        (no device allocation in the call)."""
        self._check(self.lib.hofv_jvp_noalloc(self.h, self._v(u), self._v(Ru), self._v(v), self._v(Jv),
                                              float(eps), _stream(stream)))

    def nej_apply(self, v, out, stream=None):
        """out = A v for the near-exact Jacobian A (linear elastic law)."""
        self._check(self.lib.hofv_nej_apply(self.h, self._v(v), self._v(out), _stream(stream)))

    def precond_apply(self, r, z, n_sweeps=2, learned=False, stream=None):
        self._check(self.lib.hofv_precond_apply(self.h, self._v(r), self._v(z), int(n_sweeps), int(bool(learned)),
                                                _stream(stream)))

    def fgmres_solve(self, u, Ru, rhs, x, restart=30, max_iters=1000, rtol=1e-6, n_sweeps=2, learned=False,
                     stream=None, check=True, side=0, gs_passes=0, graphs=0):
        o = L.KrylovOpts(restart, max_iters, rtol, n_sweeps, int(bool(learned)), int(side), int(gs_passes),
                         int(graphs))
        s = L.KrylovStats()
        st = self.lib.hofv_fgmres_solve(self.h, self._v(u), self._v(Ru), self._v(rhs), self._v(x), C.byref(o),
                                        C.byref(s), _stream(stream))
        if check or st not in (L.HOFV_OK, -5):
            self._check(st)
        return {k: getattr(s, k) for k, _ in L.KrylovStats._fields_}

    @staticmethod
    def _newton_opts(tol, eta, max_newton, n_increments, max_line_search, restart, max_krylov, n_sweeps, learned,
                     forcing, predictor, side=0, gs_passes=0, graphs=0):
        return L.NewtonOpts(tol, eta, max_newton, n_increments, max_line_search,
                            L.KrylovOpts(restart, max_krylov, eta, n_sweeps, int(bool(learned)), int(side),
                                         int(gs_passes), int(graphs)),
                            int(forcing), int(predictor))

    def newton_solve(self, u, tol=1e-8, eta=1e-4, max_newton=50, n_increments=1, max_line_search=10,
                     restart=30, max_krylov=2000, n_sweeps=2, learned=False, stream=None, check=True,
                     forcing=0, predictor=0, side=0, gs_passes=0, graphs=0):
        o = self._newton_opts(tol, eta, max_newton, n_increments, max_line_search, restart, max_krylov, n_sweeps,
                              learned, forcing, predictor, side, gs_passes, graphs)
        s = L.NewtonStats()
        st = self.lib.hofv_newton_solve(self.h, self._v(u), C.byref(o), C.byref(s), _stream(stream))
        if check or st not in (L.HOFV_OK, -5):
            self._check(st)
        return {k: getattr(s, k) for k, _ in L.NewtonStats._fields_}

    # ------------------------------------------------------------- dynamics
    def set_dynamics(self, rho, dt):
        """BDF2 inertia with density rho and time step dt (rho <= 0: static)."""
        self._check(self.lib.hofv_set_dynamics(self.h, float(rho), float(dt)))

    def dyn_reset(self, u_t, v_t, u_tm1=None, v_tm1=None, stream=None):
        """History of the next step; u_tm1, v_tm1 default to u_t, v_t."""
        u_tm1 = u_t if u_tm1 is None else u_tm1
        v_tm1 = v_t if v_tm1 is None else v_tm1
        self._check(self.lib.hofv_dyn_reset(self.h, self._v(u_t), self._v(u_tm1), self._v(v_t), self._v(v_tm1),
                                            _stream(stream)))

    def dyn_step(self, u, tol=1e-8, eta=1e-4, max_newton=50, max_line_search=10, restart=30, max_krylov=2000,
                 n_sweeps=2, learned=False, stream=None, check=True, forcing=0):
        """One time step from the guess in u (updated in place)."""
        o = self._newton_opts(tol, eta, max_newton, 0, max_line_search, restart, max_krylov, n_sweeps, learned,
                              forcing, 0)
        s = L.NewtonStats()
        st = self.lib.hofv_dyn_step(self.h, self._v(u), C.byref(o), C.byref(s), _stream(stream))
        if check or st not in (L.HOFV_OK, -5):
            self._check(st)
        return {k: getattr(s, k) for k, _ in L.NewtonStats._fields_}

    def host_table(self, name):
        """Copy of a setup table of a host_only context (numpy, flat)."""
        n = C.c_int64()
        eb = C.c_int32()
        data = C.c_void_p()
        self._check(self.lib.hofv_host_table(self.h, name.encode(), C.byref(n), C.byref(eb), C.byref(data)))
        dtype = {("face_coef", 8): np.float64}.get((name, eb.value))
        if dtype is None:
            dtype = {2: np.uint16, 4: np.int32, 8: np.float64}[eb.value]
            if name in ("pc_dinv", "pc_a", "nn_wf", "nn_wb", "nn_bflag"):
                dtype = np.float32
        buf = (C.c_char * (n.value * eb.value)).from_address(data.value) if n.value else b""
        return np.frombuffer(bytes(buf), dtype=dtype).copy()

    # -------------------------------------------------------------- timing
    def set_timing(self, enable, only=None):
        """Per-kernel HIP events on (resets the record) or off; only = a kernel
        name times that kernel's launches alone."""
        if enable and only:
            self._check(self.lib.hofv_set_timing_only(self.h, only.encode()))
        else:
            self._check(self.lib.hofv_set_timing(self.h, int(bool(enable))))

    def kernel_time(self, name):
        ms = C.c_double()
        n = C.c_int64()
        self._check(self.lib.hofv_kernel_time(self.h, name.encode(), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def kernel_bytes(self, name):
        b = C.c_double()
        self._check(self.lib.hofv_kernel_bytes(self.h, name.encode(), C.byref(b)))
        return b.value


class Model:
    """The learned preconditioner correction (hofv_nn) on the current device."""

    def __init__(self, seed=0):
        self.lib = L.load()
        h = C.c_void_p()
        st = self.lib.hofv_nn_create(C.c_uint64(seed), C.byref(h))
        if st != L.HOFV_OK:
            raise HofvError(st, self.lib.hofv_last_error(None).decode())
        self.h = h
        self.n_params = int(self.lib.hofv_nn_param_count())

    def close(self):
        if getattr(self, "h", None):
            self.lib.hofv_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.empty(self.n_params, np.float32)
        st = self.lib.hofv_nn_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float)), self.n_params)
        if st != L.HOFV_OK:
            raise HofvError(st, self.lib.hofv_last_error(None).decode())
        return out

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, np.float32)
        st = self.lib.hofv_nn_set_params(self.h, flat.ctypes.data_as(C.POINTER(C.c_float)), flat.size)
        if st != L.HOFV_OK:
            raise HofvError(st, self.lib.hofv_last_error(None).decode())

    def save(self, path):
        st = self.lib.hofv_nn_save(self.h, str(path).encode())
        if st != L.HOFV_OK:
            raise HofvError(st, self.lib.hofv_last_error(None).decode())

    def load(self, path):
        st = self.lib.hofv_nn_load(self.h, str(path).encode())
        if st != L.HOFV_OK:
            raise HofvError(st, self.lib.hofv_last_error(None).decode())


class PairSet:
    """Training pairs (r, e), J e = r, on one context's mesh (hofv_pairset)."""

    def __init__(self, ctx, capacity):
        self.lib = ctx.lib
        self.ctx = ctx  # the set must not outlive its context
        h = C.c_void_p()
        ctx._check(self.lib.hofv_pairset_create(ctx.h, int(capacity), C.byref(h)))
        self.h = h
        self.capacity = int(capacity)

    def close(self):
        if getattr(self, "h", None):
            self.lib.hofv_pairset_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        n = C.c_int32()
        self.lib.hofv_pairset_data(self.h, C.byref(n), None, None)
        return n.value

    def tensors(self, stream=None):
        """Copies of (r, e) as torch tensors [n_pairs, dim, n_cells]."""
        import torch
        n = len(self)
        r = torch.empty((n, self.ctx.dim, self.ctx.n_cells), dtype=torch.float64, device="cuda")
        e = torch.empty_like(r)
        if n:
            self.ctx._check(self.lib.hofv_pairset_copy(self.h, 0, n, _ptr(r), _ptr(e), _stream(stream)))
        return r, e


def _ctx_nn_methods():
    def attach(self, model):
        self._check(self.lib.hofv_nn_attach(self.h, model.h if model is not None else None))
        self._model = model

    def nn_train_step(self, model, r, e, n_sweeps=2, lr=1e-3, stream=None):
        """r, e: device tensors [n_pairs, dim, n_cells] float64."""
        loss = C.c_double()
        n = int(r.shape[0]) * self.dim * self.n_cells
        self._check(self.lib.hofv_nn_train_step(self.h, model.h, _ptr(r, n), _ptr(e, n), int(r.shape[0]),
                                                int(n_sweeps), float(lr), C.byref(loss), _stream(stream)))
        return loss.value

    def nn_gradient(self, model, r, zaj, e, stream=None):
        g = np.empty(model.n_params, np.float32)
        loss = C.c_double()
        self._check(self.lib.hofv_nn_gradient(self.h, model.h, self._v(r), self._v(zaj), self._v(e),
                                              g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss),
                                              _stream(stream)))
        return loss.value, g

    def nn_forward(self, model, r, zaj, z, stream=None):
        self._check(self.lib.hofv_nn_forward(self.h, model.h, self._v(r), self._v(zaj), self._v(z), _stream(stream)))

    def harvest_pairs(self, pairs, u, n_starts=0, length=0, newton_steps=0, seed=0, starts=None, rtol=1e-8,
                      restart=30, max_iters=3000, n_sweeps=2, stream=None):
        """Appends Krylov-type and Newton pairs at state u to the PairSet `pairs`;
        starts (optional) [n_starts, dim, n_cells] device tensor of start vectors."""
        o = L.HarvestOpts(int(n_starts), int(length), int(newton_steps), C.c_uint64(int(seed)), float(rtol),
                          int(restart), int(max_iters), int(n_sweeps))
        sp = None if starts is None else _ptr(starts, int(n_starts) * self.dim * self.n_cells)
        self._check(self.lib.hofv_harvest_pairs(self.h, self._v(u), sp, C.byref(o), pairs.h, _stream(stream)))

    for f in (attach, nn_train_step, nn_gradient, nn_forward, harvest_pairs):
        setattr(Context, f.__name__, f)


def nn_train(model, pair_sets, epochs=20, lr=1e-3, batch=4, n_sweeps=2, seed=0, stream=None):
    """hofv_nn_train over the PairSets; returns (stats dict, mean loss per epoch)."""
    lib = model.lib
    sets = (C.c_void_p * len(pair_sets))(*[p.h.value for p in pair_sets])
    hist = (C.c_double * int(epochs))()
    o = L.TrainOpts(int(epochs), int(batch), float(lr), int(n_sweeps), C.c_uint64(int(seed)),
                    C.cast(hist, C.POINTER(C.c_double)))
    s = L.TrainStats()
    st = lib.hofv_nn_train(model.h, len(pair_sets), sets, C.byref(o), C.byref(s), _stream(stream))
    if st != L.HOFV_OK:
        msg = lib.hofv_last_error(pair_sets[0].ctx.h).decode() or lib.hofv_last_error(None).decode()
        raise HofvError(st, msg)
    return {k: getattr(s, k) for k, _ in L.TrainStats._fields_}, list(hist)


_ctx_nn_methods()


def context_for(problem, fold_quadrature=True, host_only=False, precond_levels=1, progress=None):
    """Create and set up a Context for a problem description (mesh, orders,
    material, loads as point functions), evaluating the loads at the library's
    boundary and volume quadrature points.  progress(stage) is called after
    each stage when given."""
    note = progress or (lambda stage: None)
    ctx = Context(problem.mesh.dim, problem.p, problem.n_plus, problem.n_gauss, problem.material, problem.mu,
                  problem.lam, problem.alpha, problem.k_weight, problem.ghost_weight, problem.stencil_quantum,
                  fold_quadrature, host_only, precond_levels, problem.face_rule, getattr(problem, "stencil_grow", 0))
    m = problem.mesh
    if hasattr(m, "face_cells"):
        ctx.set_mesh_poly(m.verts, m.face_ptr, m.face_verts, m.face_cells, m.n_cells)
    else:
        ctx.set_mesh(m.verts, m.cells)
    note("mesh")
    cen, nor, qp = ctx.boundary_faces()
    D = problem.mesh.dim
    loads = problem.loads
    nb, nq = qp.shape[0], qp.shape[1]
    types = loads.bc_type(cen, nor) if nb else np.zeros(0, np.int32)
    ubq = loads.u_b(qp.reshape(-1, D)).reshape(nb, nq, D) if nb else None
    ubc = loads.u_b(cen) if nb else None
    tq = loads.traction(qp.reshape(-1, D), np.repeat(nor, nq, axis=0)).reshape(nb, nq, D) if nb else None
    ctx.set_bc(types, ubq, ubc, tq)
    note("boundary conditions")
    vq, _ = ctx.volume_qpoints_csr()
    ctx.set_body_force(loads.body(vq))
    note("body force")
    ctx.setup()
    note("setup")
    return ctx
