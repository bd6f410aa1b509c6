"""Thin Python binding over the C ABI (argument marshalling only).

Host arrays are numpy float64/int64; device arrays are contiguous float64
torch tensors on the current HIP device.  Every computation happens inside
libdgmg.so; nothing here falls back to Python or CPU arithmetic.
"""
import ctypes as C

import numpy as np

from . import _ffi as F

MODELS = {"fhn": 0, "ap": 1, "bo": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}
TOL_MODES = {"rel_r0": 0, "rel_b": 1, "abs": 2}
LAYOUTS = {"auto": 0, "tile_ell": 1, "axis_ell": 2, "matrix_free": 3, "axis_ell_dense": 4}
JACOBI = {"point": 0, "cell_block": 1}


def _dptr(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(F.dp)


def _iptr(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(F.i64p)


def _dev(t):
    """Device pointer of a torch tensor (float64, contiguous, on the GPU)."""
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 GPU tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Hierarchy:
    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep

    @property
    def handle(self):
        return self._h

    def n_levels(self):
        n = C.c_int32()
        F.check(F.lib().dgmg_hierarchy_info(self._h, 0, C.byref(n), None))
        return n.value

    def n_entities(self, level):
        n = C.c_int64()
        F.check(F.lib().dgmg_hierarchy_info(self._h, level, None, C.byref(n)))
        return n.value

    def parents(self, level):
        out = np.empty(self.n_entities(level), dtype=np.int64)
        F.check(F.lib().dgmg_hierarchy_parents(self._h, level, out.ctypes.data_as(F.i64p)))
        return out

    def boxes(self, level, dim):
        """dgmg_hierarchy_boxes: (lo, hi) of every entity of `level`."""
        lo = np.empty((self.n_entities(level), dim))
        hi = np.empty_like(lo)
        F.check(F.lib().dgmg_hierarchy_boxes(self._h, level, lo.ctypes.data_as(F.dp),
                                             hi.ctypes.data_as(F.dp)))
        return lo, hi

    def __del__(self):
        if getattr(self, "_h", None):
            F.lib().dgmg_destroy_hierarchy(self._h)
            self._h = None


def build_hierarchy(xyz, cell_vtx, n_levels, method="grid", grid_bins=None,
                    fanout=8, user_parents=None):
    """dgmg_build_hierarchy: nested agglomerates of a quad/hex mesh."""
    xyz, xp = _dptr(xyz)
    cells, cp = _iptr(cell_vtx)
    m = F.Mesh(xyz.shape[1], xyz.shape[0], xp, cells.shape[0], cp)
    o = F.AggloOpts()
    o.n_levels = n_levels
    o.method = {"grid": 0, "rtree_str": 1, "user": 2}[method]
    o.rtree_fanout = fanout
    keep = [xyz, cells]
    if grid_bins is not None:
        for l, bins in enumerate(grid_bins):
            for k, v in enumerate(bins):
                o.grid_bins[l][k] = int(v)
    if user_parents is not None:
        arrs = [np.ascontiguousarray(a, dtype=np.int64) for a in user_parents]
        ptrs = (F.i64p * len(arrs))(*[a.ctypes.data_as(F.i64p) for a in arrs])
        o.user_parents = ptrs
        keep += [arrs, ptrs]
    h = C.c_void_p()
    F.check(F.lib().dgmg_build_hierarchy(C.byref(m), C.byref(o), C.byref(h)))
    return Hierarchy(h, keep=None)


class TorchAllocator:
    """dgmg_allocator backed by torch's caching allocator on the current
    device: every block the library asks for is a uint8 tensor kept alive
    until the library frees it.  Marshalling only; the memory is used by the
    library's kernels."""

    def __init__(self):
        import torch
        self._torch = torch
        self.live = {}

        def _alloc(ctx, nbytes):
            try:
                t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device="cuda")
            except RuntimeError:
                return None
            p = (t.data_ptr() + 255) // 256 * 256
            self.live[p] = t
            return p

        def _free(ctx, ptr):
            self.live.pop(ptr, None)

        self._c_alloc = F.ALLOC_FN(_alloc)
        self._c_free = F.FREE_FN(_free)
        self.struct = F.Allocator(self._c_alloc, self._c_free, None)

    @property
    def live_bytes(self):
        return sum(t.numel() for t in self.live.values())


class Solver:
    def __init__(self, handle, keep=None):
        self._s = handle
        self._keep = keep   # objects the library calls back into (allocator)

    @property
    def handle(self):
        return self._s

    def info(self):
        i = F.SolverInfo()
        F.check(F.lib().dgmg_get_info(self._s, C.byref(i)))
        L = i.n_levels
        return dict(dim=i.dim, p=i.p, b=i.b, n_levels=L, precision=i.precision,
                    model=i.model, n_gates=i.n_gates, n_dofs=i.n_dofs,
                    n_cells=list(i.n_cells[:L]), n_faces=list(i.n_faces[:L]),
                    lam_lo=list(i.lam_lo[:L]), lam_hi=list(i.lam_hi[:L]),
                    op_complexity=i.op_complexity,
                    t_setup=dict(assembly=i.t_assembly, hierarchy=i.t_hierarchy,
                                 transfer=i.t_transfer, galerkin=i.t_galerkin,
                                 smoother=i.t_smoother, coarse=i.t_coarse,
                                 upload=i.t_upload),
                    device_bytes=i.device_bytes,
                    fine_layout=_LAYOUT_NAMES.get(i.fine_layout, "none"),
                    level_layout=[_LAYOUT_NAMES.get(v, "none") for v in i.level_layout[:L]],
                    prolong_types=list(i.prolong_types[:L]),
                    level_grouped=[bool(v) for v in i.level_grouped[:L]],
                    sparse_faces=bool(i.sparse_faces))

    def export_level(self, level, blocks=True):
        """Host copies of a level's FP64 operator and transfer blocks
        (blocks=False: the prolongation, parents and face list only)."""
        inf = self.info()
        b = inf["b"]
        n = inf["n_cells"][level]
        nf = inf["n_faces"][level]
        diag = np.empty((n, b, b)) if blocks else None
        fc = np.empty((nf, 2), dtype=np.int64)
        fb = np.empty((nf, b, b)) if blocks else None
        last = level == inf["n_levels"] - 1
        P = None if last else np.empty((n, b, b))
        par = None if last else np.empty(n, dtype=np.int64)
        F.check(F.lib().dgmg_export_level(
            self._s, level, None if diag is None else diag.ctypes.data_as(F.dp),
            fc.ctypes.data_as(F.i64p), None if fb is None else fb.ctypes.data_as(F.dp),
            None if P is None else P.ctypes.data_as(F.dp),
            None if par is None else par.ctypes.data_as(F.i64p)))
        return dict(diag=diag, face_cells=fc, face_blocks=fb, P=P, parents=par)

    def __del__(self):
        if getattr(self, "_s", None):
            F.lib().dgmg_destroy_solver(self._s)
            self._s = None


_LAYOUT_NAMES = {1: "tile_ell", 2: "axis_ell", 3: "matrix_free"}


def setup_levels(hier, p, D_cell, chi, Cm, dt, model, params, penalty=("paper",),
                 bdf=2, cell_scale=None, precision="fp64", cheb_degree=3,
                 cheb_sweeps=3, lanczos_steps=20, lam_safety=1.2,
                 smooth_range=20.0, lam_override=None, device_setup=True, adjoint=False,
                 max_rhs=1, mfma=False, fine_layout="auto", setup="host", allocator=None,
                 jacobi="point"):
    """dgmg_setup_levels: assembly, Galerkin hierarchy, smoother, coarse factor.
    setup = "device" computes the assembly, prolongations, Galerkin products and
    Lanczos estimates on the GPU, "host" on the CPU.  allocator: None (the
    library uses hipMalloc), "torch" or a TorchAllocator (device memory from
    torch's caching allocator).  jacobi: "point" (the diagonal) or
    "cell_block" (the cells' inverted diagonal blocks) in the smoother."""
    if setup not in ("host", "device"):
        raise ValueError("setup must be 'host' or 'device'")
    if jacobi not in JACOBI:
        raise ValueError("jacobi must be 'point' or 'cell_block'")
    d = F.Disc(p, 0 if penalty[0] == "paper" else 1,
               float(penalty[1]) if len(penalty) > 1 else 0.0)
    D_cell, Dp = _dptr(D_cell)
    params, pp = _dptr(params)
    keep = [D_cell, params]
    sp = None
    if cell_scale is not None:
        cs, sp = _dptr(cell_scale)
        keep.append(cs)
    ph = F.Physics(chi, Cm, dt, bdf, Dp, sp, MODELS[model], len(params), pp)
    lo = None
    if lam_override is not None:
        lam, lo = _dptr(np.asarray(lam_override, dtype=np.float64).ravel())
        keep.append(lam)
    if allocator == "torch":
        allocator = TorchAllocator()
    ap = None
    if allocator is not None:
        if not isinstance(allocator, TorchAllocator):
            raise ValueError("allocator must be None, 'torch' or a TorchAllocator")
        ap = C.pointer(allocator.struct)
    mg = F.MGOpts(cheb_degree, cheb_sweeps, lanczos_steps, lam_safety, smooth_range,
                  lo, PRECISIONS[precision], 1 if device_setup else 0, 1 if adjoint else 0,
                  int(max_rhs), 1 if mfma else 0, LAYOUTS[fine_layout],
                  1 if setup == "device" else 0, ap, JACOBI[jacobi])
    s = C.c_void_p()
    F.check(F.lib().dgmg_setup_levels(hier.handle, C.byref(d), C.byref(ph), C.byref(mg),
                                      C.byref(s)))
    return Solver(s, keep=allocator)


def _pcg_opts(tol, tol_mode, max_it, flexible):
    return F.PCGOpts(tol, TOL_MODES[tol_mode], max_it, 1 if flexible else 0)


def _stats(st, rc):
    return dict(its=st.its, converged=bool(st.converged), r0=st.r0, rfin=st.rfin,
                rc=rc)


def pcg_solve(solver, b, x, tol=1e-8, tol_mode="rel_r0", max_it=500, flexible=False,
              stream=None):
    """dgmg_pcg_solve: x <- A_0^-1 b by V-cycle PCG, warm-started from x."""
    st = F.PCGStats()
    o = _pcg_opts(tol, tol_mode, max_it, flexible)
    rc = F.check(F.lib().dgmg_pcg_solve(solver.handle, _dev(b), _dev(x), C.byref(o),
                                        C.byref(st), _stream(stream)))
    return _stats(st, rc)


def pcg_solve_noalloc(solver, b, x, tol=1e-8, tol_mode="rel_r0", max_it=500, flexible=False,
                      stream=None):
    """dgmg_pcg_solve_noalloc: pcg_solve with the reduction scratch in the
    library's static per-GPU array (no device allocation during the call;
    overlapping calls on one GPU race)."""
    st = F.PCGStats()
    o = _pcg_opts(tol, tol_mode, max_it, flexible)
    rc = F.check(F.lib().dgmg_pcg_solve_noalloc(solver.handle, _dev(b), _dev(x), C.byref(o),
                                                C.byref(st), _stream(stream)))
    return _stats(st, rc)


def pcg_solve_multi(solver, b, x, tol=1e-8, tol_mode="rel_r0", max_it=500, flexible=False,
                    stream=None):
    """dgmg_pcg_solve_multi: MULTI_RHS independent solves; b, x are [N, MULTI_RHS]
    column-minor device tensors.  Returns one stats dict per column."""
    st = (F.PCGStats * F.MULTI_RHS)()
    o = _pcg_opts(tol, tol_mode, max_it, flexible)
    rc = F.check(F.lib().dgmg_pcg_solve_multi(solver.handle, F.MULTI_RHS, _dev(b), _dev(x),
                                              C.byref(o), st, _stream(stream)))
    return [_stats(st[c], rc) for c in range(F.MULTI_RHS)]


def set_phase_timing(solver, on=True):
    """dgmg_set_phase_timing: record HIP events at the phase boundaries of
    every following time_step (for per-step logs; not for timed runs)."""
    F.check(F.lib().dgmg_set_phase_timing(solver.handle, 1 if on else 0))


def step_phase_ms(solver):
    """dgmg_step_phase_ms: the last timed step's ionic update, load vector and
    PCG solve durations in ms (waits for the step's final event)."""
    ms = (C.c_double * 3)()
    F.check(F.lib().dgmg_step_phase_ms(solver.handle, ms))
    return dict(ionic=ms[0], load_vector=ms[1], pcg=ms[2])


def ionic_step(solver, U, Uprev, W, Wprev, Wnext, g, stream=None):
    """dgmg_ionic_step: BDF2 gate update at U* and nodal ionic current."""
    F.check(F.lib().dgmg_ionic_step(solver.handle, _dev(U), _dev(Uprev), _dev(W),
                                    _dev(Wprev), _dev(Wnext), _dev(g), _stream(stream)))


class State:
    """Caller-owned device state (U_n, U_{n-1}, W_n, W_{n-1}, g workspace)."""

    def __init__(self, U, Uprev, W, Wprev, g):
        self.U, self.Uprev, self.W, self.Wprev, self.g = U, Uprev, W, Wprev, g

    def _struct(self):
        return F.State(self.U.data_ptr(), self.Uprev.data_ptr(), self.W.data_ptr(),
                       self.Wprev.data_ptr(), self.g.data_ptr())

    def save(self, path, **meta):
        """Checkpoint of the step state (U_n, U_{n-1}, W_n, W_{n-1}) with any
        caller metadata (time, step index) via torch.save; a time step is a
        pure function of this state, so load() resumes a run bit for bit."""
        import torch
        torch.save({"U": self.U.cpu(), "Uprev": self.Uprev.cpu(), "W": self.W.cpu(),
                    "Wprev": self.Wprev.cpu(), "meta": meta}, path)

    @classmethod
    def load(cls, path, device="cuda"):
        """(State, meta) from a save() file; the g workspace is fresh."""
        import torch
        d = torch.load(path, weights_only=True)
        to = lambda t: t.to(device).contiguous()
        st = cls(to(d["U"]), to(d["Uprev"]), to(d["W"]), to(d["Wprev"]),
                 torch.empty_like(d["U"], device=device))
        return st, d["meta"]

    def _adopt(self, s):
        # the library rotated the pointer pairs: follow it
        if s.U != self.U.data_ptr():
            self.U, self.Uprev = self.Uprev, self.U
        if s.W != self.W.data_ptr():
            self.W, self.Wprev = self.Wprev, self.W


def time_step(solver, state, t_next, iapp=None, tol=1e-8, tol_mode="rel_r0",
              max_it=500, flexible=False, stream=None):
    """dgmg_time_step: ionic update, ICI load vector, warm-started PCG."""
    for t in (state.U, state.Uprev, state.W, state.Wprev, state.g):
        _dev(t)
    s = state._struct()
    st = F.PCGStats()
    o = _pcg_opts(tol, tol_mode, max_it, flexible)
    rc = F.check(F.lib().dgmg_time_step(solver.handle, C.byref(s), t_next, _dev(iapp),
                                        C.byref(o), C.byref(st), _stream(stream)))
    state._adopt(s)
    return _stats(st, rc)


def time_step_multi(solver, state, t_next, iapp=None, tol=1e-8, tol_mode="rel_r0",
                    max_it=500, flexible=False, stream=None):
    """dgmg_time_step_multi: MULTI_RHS independent simulations; every state
    tensor holds MULTI_RHS columns (column-minor)."""
    for t in (state.U, state.Uprev, state.W, state.Wprev, state.g):
        _dev(t)
    s = state._struct()
    st = (F.PCGStats * F.MULTI_RHS)()
    o = _pcg_opts(tol, tol_mode, max_it, flexible)
    rc = F.check(F.lib().dgmg_time_step_multi(solver.handle, F.MULTI_RHS, C.byref(s), t_next,
                                              _dev(iapp), C.byref(o), st, _stream(stream)))
    state._adopt(s)
    return [_stats(st[c], rc) for c in range(F.MULTI_RHS)]


def apply_multi(solver, level, x, y, precision="fp64", stream=None):
    """dgmg_apply_multi: Y = A_level X on MULTI_RHS column-minor columns."""
    F.check(F.lib().dgmg_apply_multi(solver.handle, level, PRECISIONS[precision], F.MULTI_RHS,
                                     _dev(x), _dev(y), _stream(stream)))


def vcycle_multi(solver, r, z, stream=None):
    """dgmg_vcycle_multi: one V-cycle on each of MULTI_RHS columns."""
    F.check(F.lib().dgmg_vcycle_multi(solver.handle, F.MULTI_RHS, _dev(r), _dev(z),
                                      _stream(stream)))


def apply(solver, level, x, y, precision="fp64", stream=None):
    """dgmg_apply: y = A_level x with the FP64 or FP32 level copy."""
    F.check(F.lib().dgmg_apply(solver.handle, level, PRECISIONS[precision], _dev(x),
                               _dev(y), _stream(stream)))


def vcycle(solver, r, z, stream=None):
    """dgmg_vcycle: z = B r (one V-cycle)."""
    F.check(F.lib().dgmg_vcycle(solver.handle, _dev(r), _dev(z), _stream(stream)))


def mass_apply(solver, f, b, stream=None):
    """dgmg_mass_apply: b = M f (cellwise mass blocks)."""
    F.check(F.lib().dgmg_mass_apply(solver.handle, _dev(f), _dev(b), _stream(stream)))


KERNEL_KINDS = {"cheb_step": 0, "residual": 1, "apply": 2, "restrict": 3, "prolong": 4,
                "coarse": 5}


def profile_begin(solver, kind, level=0):
    """Start HIP-event timing of every launch of one kernel kind on one level."""
    F.check(F.lib().dgmg_profile_begin(solver.handle, KERNEL_KINDS[kind], level))


def profile_end(solver):
    """(launches, total_ms) of the kernel timed since profile_begin."""
    n = C.c_int64()
    ms = C.c_double()
    F.check(F.lib().dgmg_profile_end(solver.handle, C.byref(n), C.byref(ms)))
    return n.value, ms.value


def kernel_bench(solver, kind="cheb_step", level=0, reps=200, nrhs=1, stream=None):
    """Average duration in ms of back-to-back launches of one smoother kernel."""
    ms = C.c_double()
    F.check(F.lib().dgmg_kernel_bench(solver.handle, KERNEL_KINDS[kind], level, nrhs, reps,
                                      _stream(stream), C.byref(ms)))
    return ms.value


def set_sensors(solver, cells, ref):
    """dgmg_set_sensors: point-evaluation functionals (cell, reference point)."""
    cells, cp = _iptr(cells)
    ref, rp = _dptr(ref)
    F.check(F.lib().dgmg_set_sensors(solver.handle, len(cells), cp, rp))


def sensor_misfit(solver, U, target, Ubar, loss, stream=None):
    """dgmg_sensor_misfit: loss += |E U - target|^2; Ubar += 2 E^T (E U - target)."""
    F.check(F.lib().dgmg_sensor_misfit(solver.handle, _dev(U), _dev(target), _dev(Ubar),
                                       _dev(loss), _stream(stream)))


def adjoint_step(solver, U, Uprev, W, Wprev, lam, Wbar_in, Ubar, Uprevbar, Wbar, Wprevbar,
                 stream=None):
    """dgmg_adjoint_step: reverse of the ionic update and load vector of a step."""
    F.check(F.lib().dgmg_adjoint_step(solver.handle, _dev(U), _dev(Uprev), _dev(W), _dev(Wprev),
                                      _dev(lam), _dev(Wbar_in), _dev(Ubar), _dev(Uprevbar),
                                      _dev(Wbar), _dev(Wprevbar), _stream(stream)))


def grad_accumulate(solver, lam, U, grad, stream=None):
    """dgmg_grad_accumulate: grad_K -= lambda^T dA/ds_K U."""
    F.check(F.lib().dgmg_grad_accumulate(solver.handle, _dev(lam), _dev(U), _dev(grad),
                                         _stream(stream)))
