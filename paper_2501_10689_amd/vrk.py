"""ctypes binding of libvrk.so (include/vrk.h): argument marshalling only.

Every step of the precoding path runs in the HIP kernels of libvrk.so;
torch supplies device memory and the stream. There is no CPU fallback: if
the library is not built, importing the entry points raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvrk.so")

VARIANTS = {"grk": 0, "ahk": 1, "vr_ogrk": 2, "vr_oahk": 3}
SELECT = {"baiwu": 0, "residual": 1, "max": 2, "energy": 3, "uniform": 4}
DTYPES = {"c64": 0, "c128": 1}
ENGINES = {"auto": 0, "vector": 1, "mfma": 2}
SCHEDULES = {"auto": 0, "gather": 1, "colour": 2}
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "workspace", 4: "HIP error", 5: "call order"}
F_CONVERGED, F_NONFINITE, F_MAXITER = 1, 2, 4
Q_PERM, Q_FSET, Q_COLOUR, Q_XOFF, Q_XIDX, Q_ENGINE, Q_TILES, Q_GRAD = range(8)


class Problem(C.Structure):
    _fields_ = [("nt", C.c_int32), ("k", C.c_int32), ("xi", C.c_double),
                ("H", C.c_void_p), ("ldh", C.c_int64),
                ("vr_start", C.c_void_p), ("vr_len", C.c_void_p),
                ("nrhs", C.c_int32),
                ("S", C.c_void_p), ("lds", C.c_int64),
                ("X", C.c_void_p), ("ldx", C.c_int64),
                ("V", C.c_void_p), ("ldv", C.c_int64),
                ("GX", C.c_void_p), ("ldgx", C.c_int64),
                ("GH", C.c_void_p), ("ldgh", C.c_int64),
                ("GS", C.c_void_p), ("ldgs", C.c_int64),
                ("gxi", C.c_void_p),
                ("vr_mask", C.c_void_p), ("n_sub", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("variant", C.c_int32), ("select", C.c_int32), ("dtype", C.c_int32),
                ("engine", C.c_int32), ("tol", C.c_double), ("max_iters", C.c_int64),
                ("seed", C.c_uint64), ("schedule", C.c_int32), ("tile_waves", C.c_int32),
                ("persistent", C.c_int32), ("wave_tiles", C.c_int32), ("check_every", C.c_int32)]


class LinkOut(C.Structure):
    _fields_ = [("E", C.c_void_p), ("lde", C.c_int64), ("rate", C.c_void_p), ("beta", C.c_void_p),
                ("noise", C.c_double)]


class VrkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("vrk status %d (%s): %s" % (status, STATUS.get(status, "?"), msg))
        self.status = status


_lib = None


def lib():
    """Load libvrk.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libvrk.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(Problem)
        vp = C.c_void_p
        L.vrk_default_options.restype = None
        L.vrk_default_options.argtypes = [C.POINTER(Options)]
        L.vrk_plan_create.restype = C.c_int
        L.vrk_plan_create.argtypes = [P, C.c_int32, C.POINTER(Options), C.POINTER(C.c_size_t),
                                      C.POINTER(vp)]
        L.vrk_plan_bind.restype = C.c_int
        L.vrk_plan_bind.argtypes = [vp, vp, C.c_size_t, vp]
        L.vrk_plan_bind_static.restype = C.c_int
        L.vrk_plan_bind_static.argtypes = [vp, vp]
        L.vrk_plan_refresh.restype = C.c_int
        L.vrk_plan_refresh.argtypes = [vp, vp]
        L.vrk_solve.restype = C.c_int
        L.vrk_solve.argtypes = [vp, vp, vp, vp, vp]
        L.vrk_solve_adjoint.restype = C.c_int
        L.vrk_solve_adjoint.argtypes = [vp, vp, vp, vp, vp]
        L.vrk_autotune.restype = C.c_int
        L.vrk_autotune.argtypes = [P, C.c_int32, C.POINTER(Options), vp, C.c_size_t, vp, C.c_char_p,
                                   C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_float)]
        L.vrk_link_metrics.restype = C.c_int
        L.vrk_link_metrics.argtypes = [vp, C.POINTER(LinkOut), vp]
        L.vrk_plan_query.restype = C.c_int64
        L.vrk_plan_query.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_int64]
        L.vrk_plan_destroy.restype = None
        L.vrk_plan_destroy.argtypes = [vp]
        L.vrk_status_string.restype = C.c_char_p
        L.vrk_status_string.argtypes = [C.c_int]
        L.vrk_last_error.restype = C.c_char_p
        L.vrk_last_error.argtypes = []
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise VrkError(st, lib().vrk_last_error().decode())


def options(variant="vr_oahk", select="baiwu", dtype="c64", engine="auto", tol=1e-5,
            max_iters=100000, seed=0, schedule="auto", tile_waves=0, persistent=0, wave_tiles=0,
            check_every=1) -> Options:
    o = Options()
    lib().vrk_default_options(C.byref(o))
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    o.select = SELECT[select] if isinstance(select, str) else int(select)
    o.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    o.engine = ENGINES[engine] if isinstance(engine, str) else int(engine)
    o.tol = float(tol)
    o.max_iters = int(max_iters)
    o.seed = int(seed)
    o.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    o.tile_waves = int(tile_waves)
    o.persistent = int(persistent)
    o.wave_tiles = int(wave_tiles)
    o.check_every = int(check_every)
    return o


def _ptr(t) -> int:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stride(t) -> int:
    return int(t.stride(0)) if t is not None and t.dim() == 2 else 0


@dataclass
class ProblemSpec:
    """One drop: device tensors (torch) and host VR arrays (numpy int32;
    vr_mask uint64 with n_sub for the subarray VR model)."""

    H: object
    vr_start: np.ndarray
    vr_len: np.ndarray
    xi: float
    S: object
    X: object
    V: object = None
    GX: object = None
    GH: object = None
    GS: object = None
    gxi: object = None
    vr_mask: object = None
    n_sub: int = 0


SCRATCH_BYTES = 64 << 20   # VRK_SCRATCH_BYTES of include/vrk.h


def _validate_spec(sp: ProblemSpec, i: int, opts: Options):
    """What the C side cannot see from raw pointers: every buffer a device
    tensor on H's device, of the plan's element type, rows contiguous
    (unit inner stride), shapes consistent with H (K x Nt) and S (B x K),
    and one VR entry per user. Raises ValueError; nothing reaches the
    library otherwise."""
    import torch
    cdt = torch.complex128 if opts.dtype == DTYPES["c128"] else torch.complex64
    H = sp.H
    if not torch.is_tensor(H) or H.dim() != 2:
        raise ValueError("problem %d: H must be a 2-D torch tensor" % i)
    K, N = int(H.shape[0]), int(H.shape[1])
    B = int(sp.S.shape[0]) if sp.S is not None else 0
    shapes = {"H": (K, N), "S": (B, K), "X": (B, N), "V": (B, K), "GX": (B, N), "GH": (K, N), "GS": (B, K)}
    for name, want in shapes.items():
        t = getattr(sp, name)
        if t is None:
            if name in ("H", "S", "X") and (name == "H" or B > 0):
                raise ValueError("problem %d: %s is required" % (i, name))
            continue
        if not torch.is_tensor(t) or not t.is_cuda:
            raise ValueError("problem %d: %s must be a device (CUDA) tensor" % (i, name))
        if t.device != H.device:
            raise ValueError("problem %d: %s is on %s, H on %s" % (i, name, t.device, H.device))
        if t.dtype != cdt:
            raise ValueError("problem %d: %s is %s, the plan computes in %s" % (i, name, t.dtype, cdt))
        if t.dim() != 2 or tuple(t.shape) != want:
            raise ValueError("problem %d: %s has shape %s, expected %s" % (i, name, tuple(t.shape), want))
        if t.numel() and (t.stride(1) != 1 or t.stride(0) < want[1]):
            raise ValueError("problem %d: %s rows must be contiguous (strides %s)" % (i, name, t.stride()))
    if sp.gxi is not None:
        g = sp.gxi
        if not torch.is_tensor(g) or not g.is_cuda or g.device != H.device or g.dtype != torch.float64 \
                or g.numel() < 1:
            raise ValueError("problem %d: gxi must be a float64 device tensor on H's device" % i)
    if len(np.atleast_1d(sp.vr_start)) != K or len(np.atleast_1d(sp.vr_len)) != K:
        raise ValueError("problem %d: vr_start and vr_len need one entry per user (K = %d)" % (i, K))
    if sp.vr_mask is not None and len(np.atleast_1d(sp.vr_mask)) != K:
        raise ValueError("problem %d: vr_mask needs one entry per user (K = %d)" % (i, K))


class Plan:
    """Owns a vrk_plan, its workspace and references to every buffer it
    records. ``probs`` is a list of ProblemSpec. With ``static=True`` no
    workspace is allocated: the plan is bound to the library's scratch array
    on the current device (vrk_plan_bind_static)."""

    def __init__(self, probs, opts: Options, device=None, stream=None, static=False):
        import torch
        self._torch = torch
        self.probs = list(probs)
        self.opts = opts
        self._keep = []
        for i, sp in enumerate(self.probs):
            _validate_spec(sp, i, opts)
        arr = (Problem * len(self.probs))()
        for i, sp in enumerate(self.probs):
            vs = np.ascontiguousarray(sp.vr_start, dtype=np.int32)
            vl = np.ascontiguousarray(sp.vr_len, dtype=np.int32)
            self._keep += [vs, vl]
            p = arr[i]
            p.k, p.nt = int(sp.H.shape[0]), int(sp.H.shape[1])
            p.xi = float(sp.xi)
            p.H, p.ldh = _ptr(sp.H), _stride(sp.H)
            p.vr_start, p.vr_len = _ptr(vs), _ptr(vl)
            p.nrhs = int(sp.S.shape[0]) if sp.S is not None else 0
            p.S, p.lds = _ptr(sp.S), _stride(sp.S)
            p.X, p.ldx = _ptr(sp.X), _stride(sp.X)
            p.V, p.ldv = _ptr(sp.V), _stride(sp.V)
            p.GX, p.ldgx = _ptr(sp.GX), _stride(sp.GX)
            p.GH, p.ldgh = _ptr(sp.GH), _stride(sp.GH)
            p.GS, p.ldgs = _ptr(sp.GS), _stride(sp.GS)
            p.gxi = _ptr(sp.gxi)
            if sp.vr_mask is not None:
                vm = np.ascontiguousarray(sp.vr_mask, dtype=np.uint64)
                self._keep.append(vm)
                p.vr_mask, p.n_sub = vm.ctypes.data, int(sp.n_sub)
        self._arr = arr
        ws = C.c_size_t(0)
        h = C.c_void_p()
        _check(lib().vrk_plan_create(arr, len(self.probs), C.byref(opts), C.byref(ws), C.byref(h)))
        self._h = h
        self.ws_bytes = int(ws.value)
        self.nrhs_total = sum(int(arr[i].nrhs) for i in range(len(self.probs)))
        self.device = device if device is not None else (self.probs[0].H.device)
        self.static = bool(static)
        if self.static:
            self.workspace, self._ws_ptr = None, None
        else:
            self.workspace = torch.empty(max(self.ws_bytes, 256) + 256, dtype=torch.uint8, device=self.device)
            off = (-self.workspace.data_ptr()) % 256
            self._ws_ptr = self.workspace.data_ptr() + off
        self.bind(stream)

    def _stream(self, stream):
        if stream is None:
            return self._torch.cuda.current_stream(self.device).cuda_stream
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)

    def bind(self, stream=None):
        if self.static:
            _check(lib().vrk_plan_bind_static(self._h, self._stream(stream)))
        else:
            _check(lib().vrk_plan_bind(self._h, self._ws_ptr, self.ws_bytes, self._stream(stream)))

    def refresh(self, stream=None):
        """Recompute what the binding derives from H (row norms, tiles, Gram
        tiles) after H changed in place; graph-capturable."""
        _check(lib().vrk_plan_refresh(self._h, self._stream(stream)))

    def stats_buffers(self):
        t = self._torch
        n = max(1, self.nrhs_total)
        return (t.zeros(n, dtype=t.int32, device=self.device),
                t.zeros(n, dtype=t.float32, device=self.device),
                t.zeros(n, dtype=t.int32, device=self.device))

    def solve(self, stream=None, stats=None):
        it, rel, fl = stats if stats is not None else (None, None, None)
        _check(lib().vrk_solve(self._h, self._stream(stream), _ptr(it), _ptr(rel), _ptr(fl)))

    def solve_adjoint(self, stream=None, stats=None):
        it, rel, fl = stats if stats is not None else (None, None, None)
        _check(lib().vrk_solve_adjoint(self._h, self._stream(stream), _ptr(it), _ptr(rel), _ptr(fl)))

    def link_metrics(self, E, rate, beta, noise, stream=None):
        """After a solve with S = I_K on every problem: the effective channels
        E[p] (K x K, the plan's complex type), per-user rates rate[p] (K,
        float64, bit/s/Hz) and beta[p] (1, float64), all device tensors;
        noise[p] (or one float for all) is sigma^2 / rho of the rate."""
        n = len(self.probs)
        noise = [float(noise)] * n if np.isscalar(noise) else [float(v) for v in noise]
        if not (len(E) == len(rate) == len(beta) == len(noise) == n):
            raise ValueError("one E, rate, beta and noise per problem")
        arr = (LinkOut * n)()
        for i in range(n):
            arr[i].E, arr[i].lde = _ptr(E[i]), _stride(E[i])
            arr[i].rate, arr[i].beta = _ptr(rate[i]), _ptr(beta[i])
            arr[i].noise = noise[i]
        _check(lib().vrk_link_metrics(self._h, arr, self._stream(stream)))

    def query(self, prob: int, what: int) -> np.ndarray:
        n = lib().vrk_plan_query(self._h, prob, what, None, 0)
        if n < 0:
            raise VrkError(1, "bad query")
        out = np.zeros(max(n, 1), dtype=np.int32)
        lib().vrk_plan_query(self._h, prob, what, out.ctypes.data, n)
        return out[:n]

    def close(self):
        if getattr(self, "_h", None):
            lib().vrk_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _problem_array(probs):
    keep = []
    arr = (Problem * len(probs))()
    for i, sp in enumerate(probs):
        vs = np.ascontiguousarray(sp.vr_start, dtype=np.int32)
        vl = np.ascontiguousarray(sp.vr_len, dtype=np.int32)
        keep += [vs, vl]
        p = arr[i]
        p.k, p.nt = int(sp.H.shape[0]), int(sp.H.shape[1])
        p.xi = float(sp.xi)
        p.H, p.ldh = _ptr(sp.H), _stride(sp.H)
        p.vr_start, p.vr_len = _ptr(vs), _ptr(vl)
        p.nrhs = int(sp.S.shape[0]) if sp.S is not None else 0
        p.S, p.lds = _ptr(sp.S), _stride(sp.S)
        p.X, p.ldx = _ptr(sp.X), _stride(sp.X)
        p.V, p.ldv = _ptr(sp.V), _stride(sp.V)
        p.GX, p.ldgx = _ptr(sp.GX), _stride(sp.GX)
        p.GH, p.ldgh = _ptr(sp.GH), _stride(sp.GH)
        p.GS, p.ldgs = _ptr(sp.GS), _stride(sp.GS)
        p.gxi = _ptr(sp.gxi)
        if sp.vr_mask is not None:
            vm = np.ascontiguousarray(sp.vr_mask, dtype=np.uint64)
            keep.append(vm)
            p.vr_mask, p.n_sub = vm.ctypes.data, int(sp.n_sub)
    return arr, keep


def autotune(probs, opts: Options, cache_path=None, reps=3, stream=None):
    """Run vrk_autotune on the batch (device timing; overwrites X and V).
    Returns (tuned Options, ms per solve)."""
    import torch
    for i, sp in enumerate(probs):
        _validate_spec(sp, i, opts)
    arr, keep = _problem_array(probs)
    o = Options()
    C.pointer(o)[0] = opts
    need = C.c_size_t(0)
    _check(lib().vrk_autotune(arr, len(probs), C.byref(o), None, 0, None, None, reps, C.byref(need), None))
    dev = probs[0].H.device
    ws = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=dev)
    ptr = ws.data_ptr() + ((-ws.data_ptr()) % 256)
    st = (torch.cuda.current_stream(dev).cuda_stream if stream is None else
          (stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)))
    ms = C.c_float(0.0)
    cp = cache_path.encode() if cache_path else None
    _check(lib().vrk_autotune(arr, len(probs), C.byref(o), ptr, int(need.value), st, cp, reps,
                              C.byref(need), C.byref(ms)))
    del keep
    return o, float(ms.value)


def host_plan(nt, k, vr_start, vr_len, xi=1.0, nrhs=0, vr_mask=None, n_sub=0, adjoint=False, **kw):
    """Plan one problem on the host only (no device memory is touched; the
    device pointers are dummies, adjoint buffers included with adjoint=True).
    For inspecting the VR plan."""
    vs = np.ascontiguousarray(vr_start, dtype=np.int32)
    vl = np.ascontiguousarray(vr_len, dtype=np.int32)
    vm = None if vr_mask is None else np.ascontiguousarray(vr_mask, dtype=np.uint64)
    p = Problem()
    if vm is not None:
        p.vr_mask, p.n_sub = vm.ctypes.data, int(n_sub)
    p.nt, p.k, p.xi = nt, k, xi
    p.H, p.ldh = 256, nt
    p.vr_start, p.vr_len = vs.ctypes.data, vl.ctypes.data
    p.nrhs = nrhs
    p.S, p.lds, p.X, p.ldx = 256, k, 256, nt
    if adjoint:
        p.GX, p.ldgx, p.GH, p.ldgh, p.GS, p.ldgs, p.gxi = 256, nt, 256, nt, 256, k, 256
    o = options(**kw)
    ws = C.c_size_t(0)
    h = C.c_void_p()
    st = lib().vrk_plan_create(C.byref(p), 1, C.byref(o), C.byref(ws), C.byref(h))
    _check(st)

    class _HP:
        def __init__(self):
            self._h, self.ws_bytes = h, int(ws.value)

        def query(self, what):
            n = lib().vrk_plan_query(self._h, 0, what, None, 0)
            out = np.zeros(max(n, 1), dtype=np.int32)
            lib().vrk_plan_query(self._h, 0, what, out.ctypes.data, n)
            return out[:n]

        def __del__(self):
            lib().vrk_plan_destroy(self._h)

    return _HP()


def precoder(H, vr_start, vr_len, xi, noise, variant="vr_oahk", select="baiwu", tol=1e-5, max_iters=100000,
             seed=0, engine="auto", vr_mask=None, n_sub=0):
    """RZF precoding matrix of one drop and its link metrics on the GPU: the
    solve on S = I_K gives X = F^T (row b the unnormalised precoder of user b);
    returns X, the effective channel E = H F on the VRs (K x K), the per-user
    spectral efficiencies (bit/s/Hz, float64, with noise = sigma^2 / rho) and
    beta = 1 / ||F||_F."""
    import torch
    K = H.shape[0]
    dtype = "c128" if H.dtype == torch.complex128 else "c64"
    S = torch.eye(K, dtype=H.dtype, device=H.device)
    X = torch.empty((K, H.shape[1]), dtype=H.dtype, device=H.device)
    E = torch.empty((K, K), dtype=H.dtype, device=H.device)
    rate = torch.empty(K, dtype=torch.float64, device=H.device)
    beta = torch.empty(1, dtype=torch.float64, device=H.device)
    o = options(variant=variant, select=select, dtype=dtype, engine=engine, tol=tol, max_iters=max_iters, seed=seed)
    plan = Plan([ProblemSpec(H, vr_start, vr_len, xi, S, X, None, vr_mask=vr_mask, n_sub=n_sub)], o)
    plan.solve()
    plan.link_metrics([E], [rate], [beta], noise)
    return X, E, rate, float(beta.cpu()[0])


def precode(H, vr_start, vr_len, S, xi, variant="vr_oahk", select="baiwu", tol=1e-5,
            max_iters=100000, seed=0, engine="auto", schedule="auto", tile_waves=0,
            return_stats=False, V=True, vr_mask=None, n_sub=0):
    """Precode the rows of S (B x K) for channel H (K x Nt) on the GPU
    (vr_mask / n_sub: the subarray VR model, with vr_start / vr_len the
    hulls of the visible subarrays).

    Returns X (B x Nt) and V (B x K) as torch tensors (and the per-RHS
    iteration counts, relative residuals and flags with return_stats)."""
    import torch
    if not H.is_cuda:
        raise ValueError("H must be a device tensor")
    dtype = "c128" if H.dtype == torch.complex128 else "c64"
    S = S.reshape(-1, H.shape[0])
    B = S.shape[0]
    X = torch.empty((B, H.shape[1]), dtype=H.dtype, device=H.device)
    Vt = torch.empty((B, H.shape[0]), dtype=H.dtype, device=H.device) if V else None
    o = options(variant=variant, select=select, dtype=dtype, engine=engine, tol=tol,
                max_iters=max_iters, seed=seed, schedule=schedule, tile_waves=tile_waves)
    plan = Plan([ProblemSpec(H, vr_start, vr_len, xi, S, X, Vt, vr_mask=vr_mask, n_sub=n_sub)], o)
    st = plan.stats_buffers()
    plan.solve(stats=st)
    if return_stats:
        return X, Vt, st
    return X, Vt
