"""Python binding of libpse.so (ctypes): argument marshalling only.

Every computation runs in the HIP library; this module converts torch device
tensors to raw pointers and checks shapes.  Importing it loads the in-tree
libpse.so and raises if it is missing -- there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, 'libpse.so')

PSE_OK, PSE_WARN_NOT_CONVERGED = 0, 1
PSE_FP64, PSE_MIXED = 0, 1
PSE_REAL, PSE_WAVE, PSE_ES_BLOCK = 1, 2, 4
PSE_STATUS_NONFINITE_POS, PSE_STATUS_PAIR_OVERFLOW = 1, 2
PSE_STEP_DEVICE = 2**64 - 1


class pse_params(ctypes.Structure):
    _fields_ = [('n', ctypes.c_int64), ('box', ctypes.c_double),
                ('radius', ctypes.c_double), ('viscosity', ctypes.c_double),
                ('kT', ctypes.c_double), ('tol', ctypes.c_double),
                ('grid', ctypes.c_int32), ('support', ctypes.c_int32),
                ('xi', ctypes.c_double), ('rcut', ctypes.c_double),
                ('precision', ctypes.c_int32), ('lanczos_maxit', ctypes.c_int32),
                ('lanczos_tol', ctypes.c_double), ('gmres_restart', ctypes.c_int32),
                ('gmres_maxit', ctypes.c_int32), ('gmres_tol', ctypes.c_double),
                ('refine_passes', ctypes.c_int32), ('graphs', ctypes.c_int32),
                ('deriv_gridding', ctypes.c_int32), ('stream', ctypes.c_void_p),
                ('async_calls', ctypes.c_int32), ('deform', ctypes.c_double * 9)]


class pse_derived(ctypes.Structure):
    _fields_ = [('grid', ctypes.c_int32), ('support', ctypes.c_int32),
                ('xi', ctypes.c_double), ('eta_s', ctypes.c_double),
                ('m', ctypes.c_double), ('h', ctypes.c_double),
                ('rcut', ctypes.c_double), ('cells', ctypes.c_int32),
                ('lanczos_maxit', ctypes.c_int32), ('gmres_restart', ctypes.c_int32),
                ('gmres_maxit', ctypes.c_int32), ('refine_passes', ctypes.c_int32),
                ('lanczos_tol', ctypes.c_double), ('gmres_tol', ctypes.c_double),
                ('deriv_gridding', ctypes.c_int32), ('lambda_max', ctypes.c_double)]


class pse_stats(ctypes.Structure):
    _fields_ = [('lanczos_iters', ctypes.c_int32), ('gmres_iters', ctypes.c_int32),
                ('refine_passes', ctypes.c_int32), ('converged', ctypes.c_int32),
                ('lanczos_change', ctypes.c_double), ('gmres_residual', ctypes.c_double),
                ('fp64_residual', ctypes.c_double), ('status', ctypes.c_int32),
                ('reserved', ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class pse_step_io(ctypes.Structure):
    _fields_ = [('psi_real', ctypes.c_void_p), ('psi_wave', ctypes.c_void_p),
                ('slip', ctypes.c_void_p), ('stresslet', ctypes.c_void_p),
                ('velocity', ctypes.c_void_p)]


class pse_kernel_stat(ctypes.Structure):
    _fields_ = [('name', ctypes.c_char_p), ('launches', ctypes.c_int64),
                ('total_ms', ctypes.c_double), ('alg_bytes', ctypes.c_double)]


class pse_request(ctypes.Structure):
    _fields_ = [('n', ctypes.c_int64), ('box', ctypes.c_double), ('radius', ctypes.c_double),
                ('viscosity', ctypes.c_double), ('kT', ctypes.c_double),
                ('tol', ctypes.c_double), ('grid', ctypes.c_int32),
                ('precision', ctypes.c_int32), ('gmres_tol', ctypes.c_double),
                ('lanczos_tol', ctypes.c_double), ('steps', ctypes.c_int32),
                ('dt', ctypes.c_double), ('seed', ctypes.c_uint64),
                ('x0', ctypes.c_void_p), ('FL', ctypes.c_void_p)]


class pse_request_info(ctypes.Structure):
    _fields_ = [('id', ctypes.c_int64), ('status', ctypes.c_int32),
                ('steps_done', ctypes.c_int32), ('bytes', ctypes.c_size_t),
                ('t_submit', ctypes.c_double), ('t_admit', ctypes.c_double),
                ('t_done', ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class pse_server_info(ctypes.Structure):
    _fields_ = [('budget', ctypes.c_size_t), ('used', ctypes.c_size_t),
                ('peak_used', ctypes.c_size_t), ('active', ctypes.c_int32),
                ('peak_active', ctypes.c_int32), ('queued', ctypes.c_int32),
                ('completed', ctypes.c_int64), ('failed', ctypes.c_int64),
                ('particle_steps', ctypes.c_double), ('elapsed', ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


EXPORTS = ('pse_derive', 'pse_footprint_bytes', 'pse_create', 'pse_destroy',
           'pse_get_derived', 'pse_mobility_apply', 'pse_mobility_apply_noalloc',
           'pse_brownian_sample',
           'pse_constrained_step', 'pse_rpy_apply', 'pse_rpy_step', 'pse_fft3d', 'pse_rfft3d',
           'pse_spread', 'pse_interpolate',
           'pse_profile', 'pse_profile_read', 'pse_server_create', 'pse_server_submit',
           'pse_server_wait', 'pse_server_result', 'pse_server_release', 'pse_server_stats',
           'pse_server_destroy', 'pse_server_error', 'pse_last_error', 'pse_set_krylov',
           'pse_synchronize', 'pse_step_graph_create', 'pse_step_graph_launch',
           'pse_step_graph_destroy')


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError(f'{path} is missing: run __graft_entry__.build() '
                           '(python -m paper_1709_06946_amd.build) first')
    # torch ships its own HIP runtime under the soname libamdhip64.so.7.  Loading
    # torch first makes the library bind to that same runtime; loading the
    # library first would map the system runtime, and torch would then start
    # a second one in the process, which finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, V, I = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int
    lib.pse_derive.argtypes = [P(pse_params), P(pse_derived)]
    lib.pse_footprint_bytes.argtypes = [P(pse_params), P(ctypes.c_size_t)]
    lib.pse_create.argtypes = [P(pse_params), P(V)]
    lib.pse_destroy.argtypes = [V]
    lib.pse_get_derived.argtypes = [V, P(pse_derived)]
    lib.pse_mobility_apply.argtypes = [V, V, V, V, ctypes.c_uint]
    lib.pse_mobility_apply_noalloc.argtypes = [P(pse_params), V, V, V, ctypes.c_uint]
    # (statistics: host memory, or device-writable memory for asynchronous handles)
    lib.pse_brownian_sample.argtypes = [V, V, V, V, ctypes.c_uint64, ctypes.c_uint64,
                                        V, V, V]
    lib.pse_constrained_step.argtypes = [V, V, V, ctypes.c_double, ctypes.c_uint64,
                                         ctypes.c_uint64, P(pse_step_io), V]
    lib.pse_rpy_apply.argtypes = [V, V, V, V, ctypes.c_uint]
    lib.pse_rpy_step.argtypes = [V, V, V, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                 P(pse_step_io), V]
    lib.pse_fft3d.argtypes = [V, V, I, I]
    lib.pse_rfft3d.argtypes = [V, V, I, I]
    lib.pse_spread.argtypes = [V, V, V, I, V]
    lib.pse_interpolate.argtypes = [V, V, V, I, V]
    lib.pse_profile.argtypes = [V, I]
    lib.pse_profile_read.argtypes = [V, P(pse_kernel_stat), I, P(I)]
    lib.pse_server_create.argtypes = [ctypes.c_size_t, I, P(V)]
    lib.pse_server_submit.argtypes = [V, P(pse_request), P(ctypes.c_int64)]
    lib.pse_server_wait.argtypes = [V, ctypes.c_int64, P(pse_request_info)]
    lib.pse_server_result.argtypes = [V, ctypes.c_int64, V, V]
    lib.pse_server_release.argtypes = [V, ctypes.c_int64]
    lib.pse_server_stats.argtypes = [V, P(pse_server_info)]
    lib.pse_server_destroy.argtypes = [V]
    lib.pse_server_error.argtypes = [V, ctypes.c_int64]
    lib.pse_server_error.restype = ctypes.c_char_p
    lib.pse_set_krylov.argtypes = [V, I, I, I, I, ctypes.c_uint64]
    lib.pse_synchronize.argtypes = [V]
    lib.pse_step_graph_create.argtypes = [V, V, V, ctypes.c_double, ctypes.c_uint64, I, V,
                                          P(V)]
    lib.pse_step_graph_launch.argtypes = [V]
    lib.pse_step_graph_destroy.argtypes = [V]
    lib.pse_last_error.argtypes = [V]
    lib.pse_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ('pse_last_error', 'pse_server_error'):
            getattr(lib, name).restype = I
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


class PSEError(RuntimeError):
    pass


def make_params(n, box, *, radius=1.0, viscosity=1.0, kT=1.0, tol=1e-3, grid=0,
                support=0, xi=0.0, rcut=0.0, precision=PSE_FP64, lanczos_maxit=0,
                lanczos_tol=0.0, gmres_restart=0, gmres_maxit=0, gmres_tol=0.0,
                refine_passes=0, graphs=0, deriv_gridding=0, stream=None, async_calls=0,
                deform=None):
    """deform: 3x3 volume-preserving lattice deformation A (lattice vectors
    are the columns of box * A), or None for the cube."""
    dv = (ctypes.c_double * 9)(*([0.0] * 9 if deform is None else
                                 [float(v) for row in deform for v in row]))
    return pse_params(int(n), float(box), float(radius), float(viscosity), float(kT),
                      float(tol), int(grid), int(support), float(xi), float(rcut),
                      int(precision), int(lanczos_maxit), float(lanczos_tol),
                      int(gmres_restart), int(gmres_maxit), float(gmres_tol),
                      int(refine_passes), int(graphs), int(deriv_gridding), stream,
                      int(async_calls), dv)


def derive(params):
    d = pse_derived()
    rc = lib().pse_derive(ctypes.byref(params), ctypes.byref(d))
    if rc != PSE_OK:
        raise PSEError(f'pse_derive: {rc}: {lib().pse_last_error(None).decode()}')
    return d


def footprint_bytes(params):
    b = ctypes.c_size_t()
    rc = lib().pse_footprint_bytes(ctypes.byref(params), ctypes.byref(b))
    if rc != PSE_OK:
        raise PSEError(f'pse_footprint_bytes: {rc}: {lib().pse_last_error(None).decode()}')
    return b.value


def mobility_apply_noalloc(params, x, q, out, parts=None):
    """out = M q by the allocation-free entry point (no handle; the library's
    static device scratch holds every buffer).  params from make_params."""
    if parts is None:
        parts = PSE_REAL | PSE_WAVE
    n = params.n
    _sync()
    rc = lib().pse_mobility_apply_noalloc(
        ctypes.byref(params), _ptr(x, (n, 3), 'x'), _ptr(q, (n, 11), 'in'),
        _ptr(out, (n, 11), 'out'), parts)
    if rc < 0:
        raise PSEError(f'pse_mobility_apply_noalloc: {rc}: '
                       f'{lib().pse_last_error(None).decode()}')
    return rc


def _ptr(t, shape=None, name='tensor', dtype='float64'):
    """Raw device pointer of a contiguous device tensor of the given dtype
    ('float64' or 'complex128'), or None.  The kernels read the memory with
    that element type, so any other dtype is refused."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f'{name} must be a torch tensor')
    want = getattr(torch, dtype)
    if t.dtype != want:
        raise TypeError(f'{name} must be {dtype}, got {t.dtype}')
    if not t.is_cuda:
        raise TypeError(f'{name} must be a device tensor')
    if not t.is_contiguous():
        raise ValueError(f'{name} must be contiguous')
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f'{name} has shape {tuple(t.shape)}, expected {tuple(shape)}')
    return t.data_ptr()


def _sync():
    """Order torch's pending work on the device before a library call (the
    library runs on its own stream and synchronizes it before returning)."""
    import torch
    torch.cuda.synchronize()


class PSE:
    """One library handle (one particle count, box and parameter set).

    async_calls=1 makes an asynchronous handle: calls only enqueue work on
    the handle's stream (pass stream=<torch.cuda.Stream>.cuda_stream to order
    it with torch's work on that stream), so they can be captured into a
    graph; step statistics go to a pinned host buffer, read by stats()."""

    def __init__(self, n, box, **kw):
        self.params = make_params(n, box, **kw)
        self.n = int(n)
        self.async_calls = bool(kw.get('async_calls', 0))
        self._stats_buf = None
        if self.async_calls:
            import torch
            self._stats_buf = torch.zeros(ctypes.sizeof(pse_stats), dtype=torch.uint8,
                                          pin_memory=True)
        h = ctypes.c_void_p()
        rc = lib().pse_create(ctypes.byref(self.params), ctypes.byref(h))
        if rc != PSE_OK:
            raise PSEError(f'pse_create: {rc}: {lib().pse_last_error(None).decode()}')
        self._h = h
        d = pse_derived()
        lib().pse_get_derived(self._h, ctypes.byref(d))
        self.derived = d

    def _check(self, rc, what):
        if rc < 0:
            raise PSEError(f'{what}: {rc}: {lib().pse_last_error(self._h).decode()}')
        return rc

    def close(self):
        if getattr(self, '_h', None):
            lib().pse_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mobility_apply(self, x, q, out, parts=PSE_REAL | PSE_WAVE):
        n = self.n
        _sync()
        return self._check(lib().pse_mobility_apply(
            self._h, _ptr(x, (n, 3), 'x'), _ptr(q, (n, 11), 'in'),
            _ptr(out, (n, 11), 'out'), parts), 'pse_mobility_apply')

    def brownian_sample(self, x, psi_real=None, psi_wave=None, seed=0, counter=0,
                        out_real=None, out_wave=None):
        n, g = self.n, self.derived.grid
        if not self.async_calls:
            _sync()
        arg, st = self._stats_arg()
        rc = self._check(lib().pse_brownian_sample(
            self._h, _ptr(x, (n, 3), 'x'), _ptr(psi_real, (n, 11), 'psi_real'),
            _ptr(psi_wave, (3, g, g, g // 2 + 1), 'psi_wave', 'complex128'), seed, counter,
            _ptr(out_real, (n, 11), 'out_real'), _ptr(out_wave, (n, 11), 'out_wave'),
            arg), 'pse_brownian_sample')
        return rc, (st.as_dict() if st is not None else None)

    def _stats_arg(self):
        """(argument, host struct): a host struct for synchronous handles, the
        pinned buffer for asynchronous ones (written by the device)."""
        if self.async_calls:
            return ctypes.c_void_p(self._stats_buf.data_ptr()), None
        st = pse_stats()
        return ctypes.cast(ctypes.pointer(st), ctypes.c_void_p), st

    def stats(self):
        """Statistics of the last asynchronous call, once the device has
        finished it (synchronises the device)."""
        import torch
        torch.cuda.synchronize()
        return pse_stats.from_buffer_copy(bytes(self._stats_buf.numpy())).as_dict()

    def constrained_step(self, x, FL=None, dt=1e-3, seed=0, step=0, psi_real=None,
                         psi_wave=None, slip=None, stresslet=None, velocity=None):
        """One step; returns (status, stats) -- stats None for asynchronous
        handles (see stats())."""
        n, g = self.n, self.derived.grid
        if not self.async_calls:
            _sync()
        io = pse_step_io(_ptr(psi_real, (n, 11), 'psi_real'),
                         _ptr(psi_wave, (3, g, g, g // 2 + 1), 'psi_wave', 'complex128'),
                         _ptr(slip, (n, 11), 'slip'), _ptr(stresslet, (n, 5), 'stresslet'),
                         _ptr(velocity, (n, 3), 'velocity'))
        arg, st = self._stats_arg()
        rc = self._check(lib().pse_constrained_step(
            self._h, _ptr(x, (n, 3), 'x'), _ptr(FL, (n, 6), 'FL'), float(dt), seed, step,
            ctypes.byref(io), arg), 'pse_constrained_step')
        return rc, (st.as_dict() if st is not None else None)

    def set_krylov(self, async_calls, lanczos_iters=1, gmres_iters=1, refine_passes=1,
                   next_step=0):
        """Switch the live handle between synchronous and asynchronous calls
        (pse_set_krylov); an asynchronous handle's statistics go to a pinned
        buffer read by stats()."""
        if async_calls and self._stats_buf is None:
            import torch
            self._stats_buf = torch.zeros(ctypes.sizeof(pse_stats), dtype=torch.uint8,
                                          pin_memory=True)
        self._check(lib().pse_set_krylov(self._h, int(async_calls), int(lanczos_iters),
                                         int(gmres_iters), int(refine_passes),
                                         int(next_step)), 'pse_set_krylov')
        self.async_calls = bool(async_calls)

    def synchronize(self):
        self._check(lib().pse_synchronize(self._h), 'pse_synchronize')

    def step_graph(self, x, FL=None, dt=1e-3, seed=0, steps=1):
        """StepGraph of `steps` captured constrained steps (asynchronous
        handle on its own stream; x updated in place by every launch)."""
        return StepGraph(self, x, FL, dt, seed, steps)

    def rpy_apply(self, x, F, out, parts=PSE_REAL | PSE_WAVE):
        """out = M_UF F (the RPY-level product; F, out of shape (N, 3))."""
        n = self.n
        _sync()
        return self._check(lib().pse_rpy_apply(
            self._h, _ptr(x, (n, 3), 'x'), _ptr(F, (n, 3), 'F'), _ptr(out, (n, 3), 'out'),
            parts), 'pse_rpy_apply')

    def rpy_step(self, x, F=None, dt=1e-3, seed=0, step=0, psi_real=None, psi_wave=None,
                 slip=None, velocity=None):
        """One unconstrained RPY-level Euler-Maruyama step (x updated in place)."""
        n, g = self.n, self.derived.grid
        if not self.async_calls:
            _sync()
        io = pse_step_io(_ptr(psi_real, (n, 3), 'psi_real'),
                         _ptr(psi_wave, (3, g, g, g // 2 + 1), 'psi_wave', 'complex128'),
                         _ptr(slip, (n, 3), 'slip'), None, _ptr(velocity, (n, 3), 'velocity'))
        arg, st = self._stats_arg()
        rc = self._check(lib().pse_rpy_step(
            self._h, _ptr(x, (n, 3), 'x'), _ptr(F, (n, 3), 'F'), float(dt), seed, step,
            ctypes.byref(io), arg), 'pse_rpy_step')
        return rc, (st.as_dict() if st is not None else None)

    def profile(self, enable):
        return self._check(lib().pse_profile(self._h, int(bool(enable))), 'pse_profile')

    def profile_read(self):
        arr = (pse_kernel_stat * 16)()
        cnt = ctypes.c_int()
        self._check(lib().pse_profile_read(self._h, arr, 16, ctypes.byref(cnt)),
                    'pse_profile_read')
        return {arr[i].name.decode(): dict(launches=arr[i].launches, total_ms=arr[i].total_ms,
                                           alg_bytes=arr[i].alg_bytes)
                for i in range(cnt.value)}

    def fft3d(self, data, direction):
        g = self.derived.grid
        _sync()
        nc = data.shape[0]
        return self._check(lib().pse_fft3d(self._h, _ptr(data, (nc, g, g, g), 'data', 'complex128'), nc,
                                           direction), 'pse_fft3d')

    def rfft3d(self, data, direction):
        """In place: real grids (nc, g, g, g) float64 <-> half spectra stored in
        the same memory (view as complex (nc, g, g, g // 2))."""
        g = self.derived.grid
        _sync()
        nc = data.shape[0]
        return self._check(lib().pse_rfft3d(self._h, _ptr(data, (nc, g, g, g), 'data'), nc,
                                            direction), 'pse_rfft3d')

    def spread(self, x, q, grids):
        n, g = self.n, self.derived.grid
        _sync()
        nc = q.shape[1]
        return self._check(lib().pse_spread(self._h, _ptr(x, (n, 3), 'x'),
                                            _ptr(q, (n, nc), 'q'), nc,
                                            _ptr(grids, (nc, g, g, g), 'grids')),
                           'pse_spread')

    def interpolate(self, x, grids, out):
        n, g = self.n, self.derived.grid
        _sync()
        nc = grids.shape[0]
        return self._check(lib().pse_interpolate(self._h, _ptr(x, (n, 3), 'x'),
                                                 _ptr(grids, (nc, g, g, g), 'grids'), nc,
                                                 _ptr(out, (n, nc), 'out')),
                           'pse_interpolate')


class StepGraph:
    """Graph-captured constrained steps of an asynchronous handle
    (pse_step_graph_*): launch() enqueues one replay on the handle's stream."""

    def __init__(self, handle, x, FL, dt, seed, steps):
        n = handle.n
        _sync()
        self.handle = handle
        self._keep = (x, FL)
        g = ctypes.c_void_p()
        handle._check(lib().pse_step_graph_create(
            handle._h, _ptr(x, (n, 3), 'x'), _ptr(FL, (n, 6), 'FL'), float(dt), seed,
            int(steps), ctypes.c_void_p(handle._stats_buf.data_ptr()), ctypes.byref(g)),
            'pse_step_graph_create')
        self._g = g

    def launch(self):
        self.handle._check(lib().pse_step_graph_launch(self._g), 'pse_step_graph_launch')

    def close(self):
        if getattr(self, '_g', None):
            lib().pse_step_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PSEServer:
    """Serving runtime: queue of independent simulations admitted onto the GPU
    by device footprint, several running at once (host numpy arrays in/out)."""

    def __init__(self, budget_bytes=0, max_active=4):
        h = ctypes.c_void_p()
        rc = lib().pse_server_create(int(budget_bytes), int(max_active), ctypes.byref(h))
        if rc != PSE_OK:
            raise PSEError(f'pse_server_create: {rc}')
        self._h = h
        self._meta = {}

    def submit(self, x0, box, *, FL=None, steps=10, dt=1e-3, seed=0, radius=1.0,
               viscosity=1.0, kT=1.0, tol=1e-3, grid=0, precision=PSE_FP64,
               gmres_tol=0.0, lanczos_tol=0.0):
        import numpy as np
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        n = x0.shape[0]
        fl = None if FL is None else np.ascontiguousarray(FL, dtype=np.float64)
        req = pse_request(n, float(box), float(radius), float(viscosity), float(kT),
                          float(tol), int(grid), int(precision), float(gmres_tol),
                          float(lanczos_tol), int(steps), float(dt), int(seed),
                          x0.ctypes.data, None if fl is None else fl.ctypes.data)
        rid = ctypes.c_int64()
        rc = lib().pse_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid))
        if rc != PSE_OK:
            raise PSEError(f'pse_server_submit: {rc}')
        self._meta[rid.value] = (n, int(steps))
        return rid.value

    def wait(self, rid):
        info = pse_request_info()
        rc = lib().pse_server_wait(self._h, int(rid), ctypes.byref(info))
        if rc < 0:
            msg = lib().pse_server_error(self._h, int(rid)).decode()
            raise PSEError(f'request {rid} failed: {rc}: {msg}')
        return info.as_dict()

    def result(self, rid):
        import numpy as np
        n, steps = self._meta[rid]
        x = np.zeros((n, 3))
        lat = np.zeros(max(steps, 1))
        rc = lib().pse_server_result(self._h, int(rid), x.ctypes.data, lat.ctypes.data)
        if rc != PSE_OK:
            raise PSEError(f'pse_server_result: {rc}')
        return x, lat[:steps]

    def release(self, rid):
        lib().pse_server_release(self._h, int(rid))
        self._meta.pop(rid, None)

    def stats(self):
        info = pse_server_info()
        lib().pse_server_stats(self._h, ctypes.byref(info))
        return info.as_dict()

    def close(self):
        if getattr(self, '_h', None):
            lib().pse_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SUPPORTED_GRIDS = sorted({2**j for j in range(3, 11)} | {3 * 2**j for j in range(2, 9)})


def grid_for(box, h_max=0.5, radius=1.0):
    """Smallest supported grid with spacing <= h_max * radius."""
    need = box / (h_max * radius)
    for g in SUPPORTED_GRIDS:
        if g >= need:
            return g
    raise ValueError(f'box {box} needs a grid above 1024')
