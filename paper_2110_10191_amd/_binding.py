"""ctypes binding of include/grmhd.h. Argument marshalling only."""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrmhd.so")

NG = 3
NVAR = 8
GRMHD_OK, GRMHD_EINVAL, GRMHD_ENOMEM, GRMHD_EDEVICE, GRMHD_EUNSUPPORTED, GRMHD_ESTATE = 0, -1, -2, -3, -4, -5
GRMHD_OPT_FLOORS, GRMHD_OPT_FIXUP = 1, 2

# every symbol include/grmhd.h declares
EXPORTED = [
    "grmhd_init", "grmhd_context_bytes", "grmhd_free", "grmhd_state_layout", "grmhd_prim_to_cons", "grmhd_cons_to_prim",
    "grmhd_get_dt", "grmhd_step", "grmhd_step_electrons", "grmhd_run_electrons", "grmhd_run", "grmhd_fill_ghosts", "grmhd_substep", "grmhd_update", "grmhd_fixup", "grmhd_speeds", "grmhd_courant_dt", "grmhd_divb", "grmhd_divb_noalloc", "grmhd_step_failures", "grmhd_strerror",
    "grmhd_last_error", "grmhd_version", "grmhd_profile", "grmhd_profile_kernels", "grmhd_profile_read",
    "grmhd_set_tiles", "grmhd_get_tiles", "grmhd_batch_create", "grmhd_batch_set_dt", "grmhd_batch_get", "grmhd_batch_step", "grmhd_batch_step_electrons",
    "grmhd_batch_free", "grmhd_batch_last_error", "grmhd_batch_profile", "grmhd_batch_profile_read",
]
KERNELS = {"ghosts": 0, "sweeps": 1, "update": 4, "fixup": 5, "electrons": 6}
NSCALAR = 2
HEAT_MODELS = {"constant": 0, "kawazura": 1, "werner": 2, "rowan": 3, "howes": 4, "sharma": 5}
TILES = {"sweep": 0, "update": 1}


class GrmhdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Problem(ctypes.Structure):
    """Mirror of ``grmhd_problem``."""
    _fields_ = [
        ("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32),
        ("coords", ctypes.c_int32),
        ("a", ctypes.c_double), ("gam", ctypes.c_double), ("cfl", ctypes.c_double),
        ("x1min", ctypes.c_double), ("x1max", ctypes.c_double),
        ("x2min", ctypes.c_double), ("x2max", ctypes.c_double),
        ("x3min", ctypes.c_double), ("x3max", ctypes.c_double),
        ("hslope", ctypes.c_double), ("poly_xt", ctypes.c_double),
        ("poly_alpha", ctypes.c_double), ("mks_smooth", ctypes.c_double),
        ("recon", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("floors", ctypes.c_int32),
        ("rho_fl", ctypes.c_double), ("u_fl", ctypes.c_double), ("sigma_max", ctypes.c_double),
        ("beta_min", ctypes.c_double), ("uorho_max", ctypes.c_double), ("gamma_max", ctypes.c_double),
    ]

    @classmethod
    def from_dict(cls, prm):
        p = cls()
        for name, _ in cls._fields_:
            if name == "bc":
                for d in range(3):
                    for s in range(2):
                        p.bc[d][s] = int(prm["bc"][d][s])
            else:
                setattr(p, name, prm[name])
        return p


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2110_10191_amd/build.py`")
    # torch's HIP runtime must be the one in the process: torch asks the loader
    # for "libamdhip64.so" and the library for "libamdhip64.so.7", so loading
    # the library first would bring in a second runtime that torch then does
    # not share. Imported first, torch's copy satisfies both names.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    sig = {
        "grmhd_init": ([ctypes.POINTER(Problem), vp, ctypes.POINTER(vp)], ctypes.c_int),
        "grmhd_free": ([vp], ctypes.c_int),
        "grmhd_context_bytes": ([ctypes.POINTER(Problem), ctypes.POINTER(i64), ctypes.POINTER(i64)], ctypes.c_int),
        "grmhd_state_layout": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)], ctypes.c_int),
        "grmhd_prim_to_cons": ([vp, vp, vp], ctypes.c_int),
        "grmhd_cons_to_prim": ([vp, vp, vp, vp, i32, ctypes.POINTER(i64)], ctypes.c_int),
        "grmhd_get_dt": ([vp, vp, dp], ctypes.c_int),
        "grmhd_step": ([vp, vp, ctypes.c_double, dp], ctypes.c_int),
        "grmhd_step_electrons": ([vp, vp, vp, ctypes.c_double, i32, ctypes.c_double, dp], ctypes.c_int),
        "grmhd_run_electrons": ([vp, vp, vp, i32, dp, i32, ctypes.c_double], ctypes.c_int),
        "grmhd_run": ([vp, vp, i32, dp], ctypes.c_int),
        "grmhd_fill_ghosts": ([vp, vp, vp], ctypes.c_int),
        "grmhd_substep": ([vp, vp, vp, vp, ctypes.c_double, i32], ctypes.c_int),
        "grmhd_speeds": ([vp, dp], ctypes.c_int),
        "grmhd_update": ([vp, vp, vp, vp, ctypes.c_double, i32, vp], ctypes.c_int),
        "grmhd_fixup": ([vp, vp, vp, i32], ctypes.c_int),
        "grmhd_courant_dt": ([vp, dp, i32, dp], ctypes.c_int),
        "grmhd_divb": ([vp, vp, dp], ctypes.c_int),
        "grmhd_divb_noalloc": ([vp, vp, dp], ctypes.c_int),
        "grmhd_step_failures": ([vp, ctypes.POINTER(i64)], ctypes.c_int),
        "grmhd_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "grmhd_last_error": ([vp], ctypes.c_char_p),
        "grmhd_version": ([], ctypes.c_int),
        "grmhd_profile": ([vp, i32], ctypes.c_int),
        "grmhd_profile_kernels": ([vp, i32], ctypes.c_int),
        "grmhd_profile_read": ([vp, i32, dp, ctypes.POINTER(i64)], ctypes.c_int),
        "grmhd_set_tiles": ([vp, i32, i32, i32], ctypes.c_int),
        "grmhd_get_tiles": ([vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)], ctypes.c_int),
        "grmhd_batch_create": ([ctypes.POINTER(vp), i32, vp, ctypes.POINTER(vp)], ctypes.c_int),
        "grmhd_batch_set_dt": ([vp, dp], ctypes.c_int),
        "grmhd_batch_get": ([vp, dp, ctypes.POINTER(i32)], ctypes.c_int),
        "grmhd_batch_step": ([vp, ctypes.POINTER(vp), ctypes.POINTER(i32), i32], ctypes.c_int),
        "grmhd_batch_step_electrons": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i32),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32), i32], ctypes.c_int),
        "grmhd_batch_free": ([vp], ctypes.c_int),
        "grmhd_batch_profile": ([vp, i32], ctypes.c_int),
        "grmhd_batch_profile_read": ([vp, i32, dp, ctypes.POINTER(i64)], ctypes.c_int),
        "grmhd_batch_last_error": ([vp], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def _check(status, ctx=None):
    if status != GRMHD_OK:
        msg = lib.grmhd_last_error(ctx).decode() or lib.grmhd_strerror(status).decode()
        raise GrmhdError(status, msg)


def _ptr(t):
    """Device pointer of a torch tensor (or an int address); None -> NULL."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ----------------------------------------------------------------- C-named calls

def grmhd_init(prm, stream=None):
    """Create a context for problem dict ``prm`` on the current device and stream."""
    p = Problem.from_dict(prm)
    out = ctypes.c_void_p()
    _check(lib.grmhd_init(ctypes.byref(p), _stream_handle(stream), ctypes.byref(out)))
    return out.value


def grmhd_context_bytes(prm):
    """(context bytes, one state's bytes) a problem needs on the device."""
    p = Problem.from_dict(prm)
    cb = ctypes.c_int64()
    sb = ctypes.c_int64()
    _check(lib.grmhd_context_bytes(ctypes.byref(p), ctypes.byref(cb), ctypes.byref(sb)))
    return cb.value, sb.value


def grmhd_free(ctx):
    _check(lib.grmhd_free(ctx))


def grmhd_state_layout(ctx):
    shape = (ctypes.c_int64 * 4)()
    strides = (ctypes.c_int64 * 4)()
    off = ctypes.c_int64()
    _check(lib.grmhd_state_layout(ctx, shape, strides, ctypes.byref(off)), ctx)
    return tuple(shape), tuple(strides), off.value


def grmhd_prim_to_cons(ctx, P, U):
    _check(lib.grmhd_prim_to_cons(ctx, _ptr(P), _ptr(U)), ctx)


def grmhd_cons_to_prim(ctx, U, P, flags=None, opts=GRMHD_OPT_FLOORS | GRMHD_OPT_FIXUP, count=True):
    nf = ctypes.c_int64(-1)
    _check(lib.grmhd_cons_to_prim(ctx, _ptr(U), _ptr(P), _ptr(flags), opts,
                                  ctypes.byref(nf) if count else None), ctx)
    return nf.value if count else None


def grmhd_get_dt(ctx, P):
    dt = ctypes.c_double()
    _check(lib.grmhd_get_dt(ctx, _ptr(P), ctypes.byref(dt)), ctx)
    return dt.value


def grmhd_step(ctx, P, dt, want_dt_next=True):
    dn = ctypes.c_double()
    _check(lib.grmhd_step(ctx, _ptr(P), float(dt), ctypes.byref(dn) if want_dt_next else None), ctx)
    return dn.value if want_dt_next else None


def grmhd_step_electrons(ctx, P, E, dt, model=0, fel=0.5, want_dt_next=True):
    """One step of P and the electron entropies E; model: a HEAT_MODELS name or value."""
    m = HEAT_MODELS[model] if isinstance(model, str) else int(model)
    dn = ctypes.c_double()
    _check(lib.grmhd_step_electrons(ctx, _ptr(P), _ptr(E), float(dt), m, float(fel),
                                    ctypes.byref(dn) if want_dt_next else None), ctx)
    return dn.value if want_dt_next else None


def grmhd_run_electrons(ctx, P, E, nsteps, dt, model=0, fel=0.5):
    """nsteps electron steps with the step size kept on the device; returns the next dt."""
    m = HEAT_MODELS[model] if isinstance(model, str) else int(model)
    d = ctypes.c_double(float(dt))
    _check(lib.grmhd_run_electrons(ctx, _ptr(P), _ptr(E), int(nsteps), ctypes.byref(d), m, float(fel)), ctx)
    return d.value


def grmhd_run(ctx, P, nsteps, dt):
    """nsteps steps with the step size kept on the device; returns the next dt."""
    d = ctypes.c_double(float(dt))
    _check(lib.grmhd_run(ctx, _ptr(P), int(nsteps), ctypes.byref(d)), ctx)
    return d.value


def grmhd_fill_ghosts(ctx, P, base=None):
    _check(lib.grmhd_fill_ghosts(ctx, _ptr(P), _ptr(base)), ctx)


def grmhd_substep(ctx, Ps, Pb, Pout, dt, want_speeds=False):
    _check(lib.grmhd_substep(ctx, _ptr(Ps), _ptr(Pb), _ptr(Pout), float(dt), 1 if want_speeds else 0), ctx)


def grmhd_update(ctx, Ps, Pb, Pout, dt, flags, want_speeds=False):
    _check(lib.grmhd_update(ctx, _ptr(Ps), _ptr(Pb), _ptr(Pout), float(dt), 1 if want_speeds else 0, _ptr(flags)), ctx)


def grmhd_fixup(ctx, P, flags, halo_sides=0):
    _check(lib.grmhd_fixup(ctx, _ptr(P), _ptr(flags), int(halo_sides)), ctx)


def grmhd_speeds(ctx):
    v = (ctypes.c_double * 3)()
    _check(lib.grmhd_speeds(ctx, v), ctx)
    return tuple(v)


def grmhd_courant_dt(ctx, speeds):
    """Courant step of a split domain from each part's (ctop_1, ctop_2, ctop_3)."""
    flat = [float(c) for part in speeds for c in part]
    arr = (ctypes.c_double * len(flat))(*flat)
    dt = ctypes.c_double()
    _check(lib.grmhd_courant_dt(ctx, arr, len(speeds), ctypes.byref(dt)), ctx)
    return dt.value


def grmhd_divb(ctx, P):
    v = ctypes.c_double()
    _check(lib.grmhd_divb(ctx, _ptr(P), ctypes.byref(v)), ctx)
    return v.value


def grmhd_divb_noalloc(ctx, P):
    v = ctypes.c_double()
    _check(lib.grmhd_divb_noalloc(ctx, _ptr(P), ctypes.byref(v)), ctx)
    return v.value


def grmhd_step_failures(ctx):
    n = ctypes.c_int64()
    _check(lib.grmhd_step_failures(ctx, ctypes.byref(n)), ctx)
    return n.value


def grmhd_strerror(status):
    return lib.grmhd_strerror(status).decode()


def grmhd_last_error(ctx=None):
    return lib.grmhd_last_error(ctx).decode()


def grmhd_version():
    return lib.grmhd_version()


def grmhd_profile(ctx, enable):
    _check(lib.grmhd_profile(ctx, 1 if enable else 0), ctx)


def grmhd_profile_kernels(ctx, kernels):
    """Bracket only these kernel classes (names or ids) while profiling is on."""
    mask = 0
    for k in kernels:
        mask |= 1 << (KERNELS[k] if isinstance(k, str) else int(k))
    _check(lib.grmhd_profile_kernels(ctx, mask), ctx)


def grmhd_profile_read(ctx, kernel):
    """(total ms, launches) of one kernel class ('sweeps', 'update', ... or its id)."""
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib.grmhd_profile_read(ctx, k, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return ms.value, n.value


def grmhd_set_tiles(ctx, which, tx, ty):
    """Block tile (tx along x1, ty along x2) of the 'sweep' or 'update' kernels."""
    w = TILES[which] if isinstance(which, str) else int(which)
    _check(lib.grmhd_set_tiles(ctx, w, int(tx), int(ty)), ctx)


def grmhd_get_tiles(ctx, which):
    w = TILES[which] if isinstance(which, str) else int(which)
    tx = ctypes.c_int32()
    ty = ctypes.c_int32()
    _check(lib.grmhd_get_tiles(ctx, w, ctypes.byref(tx), ctypes.byref(ty)), ctx)
    return tx.value, ty.value


def _bcheck(status, b=None):
    if status != GRMHD_OK:
        msg = lib.grmhd_batch_last_error(b).decode() or lib.grmhd_strerror(status).decode()
        raise GrmhdError(status, msg)


def grmhd_batch_create(ctxs, stream=None):
    arr = (ctypes.c_void_p * len(ctxs))(*ctxs)
    out = ctypes.c_void_p()
    _bcheck(lib.grmhd_batch_create(arr, len(ctxs), _stream_handle(stream), ctypes.byref(out)))
    return out.value


def grmhd_batch_set_dt(b, dts):
    arr = (ctypes.c_double * len(dts))(*[float(x) for x in dts])
    _bcheck(lib.grmhd_batch_set_dt(b, arr), b)


def grmhd_batch_get(b, n):
    dt = (ctypes.c_double * n)()
    st = (ctypes.c_int32 * n)()
    _bcheck(lib.grmhd_batch_get(b, dt, st), b)
    return list(dt), list(st)


def grmhd_batch_step(b, states, active=None, nsteps=1):
    n = len(states)
    ptrs = (ctypes.c_void_p * n)(*[_ptr(s) if s is not None else None for s in states])
    act = None if active is None else (ctypes.c_int32 * n)(*[1 if a else 0 for a in active])
    _bcheck(lib.grmhd_batch_step(b, ptrs, act, int(nsteps)), b)


def grmhd_batch_step_electrons(b, states, electrons, active=None, nsteps=1):
    """electrons: per job None (no electron heating) or (E, model, fel)."""
    n = len(states)
    ptrs = (ctypes.c_void_p * n)(*[_ptr(s) if s is not None else None for s in states])
    eptr = (ctypes.c_void_p * n)(*[_ptr(e[0]) if e is not None else None for e in electrons])
    models = (ctypes.c_int32 * n)(*[(HEAT_MODELS[e[1]] if isinstance(e[1], str) else int(e[1])) if e is not None
                                    else 0 for e in electrons])
    fels = (ctypes.c_double * n)(*[float(e[2]) if e is not None else 0.0 for e in electrons])
    act = None if active is None else (ctypes.c_int32 * n)(*[1 if a else 0 for a in active])
    _bcheck(lib.grmhd_batch_step_electrons(b, ptrs, eptr, models, fels, act, int(nsteps)), b)


def grmhd_batch_profile(b, enable):
    _bcheck(lib.grmhd_batch_profile(b, 1 if enable else 0), b)


def grmhd_batch_profile_read(b, kernel):
    """(total ms, launches) of one kernel class over batch steps since profiling began."""
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _bcheck(lib.grmhd_batch_profile_read(b, k, ctypes.byref(ms), ctypes.byref(n)), b)
    return ms.value, n.value


def grmhd_batch_free(b):
    _bcheck(lib.grmhd_batch_free(b))


def grmhd_batch_last_error(b=None):
    return lib.grmhd_batch_last_error(b).decode()


class Batch:
    """Several Sim objects (same recon and precision) advanced together."""

    def __init__(self, sims, stream=None):
        self.sims = list(sims)
        self.b = grmhd_batch_create([s.ctx for s in self.sims], stream)

    def set_dt(self, dts):
        grmhd_batch_set_dt(self.b, dts)

    def get(self):
        return grmhd_batch_get(self.b, len(self.sims))

    def step(self, states, active=None, nsteps=1, electrons=None):
        """electrons: None, or per job None / (E, model, fel) for electron heating."""
        if electrons is None:
            grmhd_batch_step(self.b, states, active, nsteps)
        else:
            grmhd_batch_step_electrons(self.b, states, electrons, active, nsteps)

    def profile(self, enable):
        grmhd_batch_profile(self.b, enable)

    def profile_read(self, kernel):
        return grmhd_batch_profile_read(self.b, kernel)

    def close(self):
        if self.b:
            grmhd_batch_free(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- convenience

class Sim:
    """A context plus helpers to move padded numpy states to and from the device.

    Host arrays use the generator layout [8, n3+6, n2+6, n1+6]; device tensors
    use the library layout [8, n3+6, n2+6, n1p] (x1 rows padded to 8 doubles).
    """

    def __init__(self, prm, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.prm = prm
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.ctx = grmhd_init(prm, stream)
        self.shape, self.strides, self.offset = grmhd_state_layout(self.ctx)

    def close(self):
        if self.ctx:
            grmhd_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty_state(self):
        return self.torch.zeros(self.shape, dtype=self.torch.float64, device=self.device)

    def empty_scalars(self):
        """Device array of the two electron-heating entropies (state strides)."""
        return self.torch.zeros((NSCALAR,) + tuple(self.shape[1:]), dtype=self.torch.float64, device=self.device)

    def to_device(self, P):
        """[nvar, n3+6, n2+6, n1+6] numpy -> padded device tensor (8 primitives
        or the 2 electron entropies)."""
        t = self.empty_state() if P.shape[0] == NVAR else self.empty_scalars()
        n1 = P.shape[-1]
        t[..., :n1] = self.torch.from_numpy(P).to(self.device)
        return t

    def to_host(self, t):
        n1 = self.prm["n1"] + 2 * NG
        return t[..., :n1].cpu().numpy()

    def interior(self, t):
        p = self.prm
        return t[:, NG:NG + p["n3"], NG:NG + p["n2"], NG:NG + p["n1"]]

    # C-call wrappers
    def prim_to_cons(self, P, U):
        grmhd_prim_to_cons(self.ctx, P, U)

    def cons_to_prim(self, U, P, flags=None, opts=GRMHD_OPT_FLOORS | GRMHD_OPT_FIXUP):
        return grmhd_cons_to_prim(self.ctx, U, P, flags, opts)

    def get_dt(self, P):
        return grmhd_get_dt(self.ctx, P)

    def step(self, P, dt, want_dt_next=True):
        return grmhd_step(self.ctx, P, dt, want_dt_next)

    def run(self, P, nsteps, dt):
        return grmhd_run(self.ctx, P, nsteps, dt)

    def step_electrons(self, P, E, dt, model=0, fel=0.5, want_dt_next=True):
        return grmhd_step_electrons(self.ctx, P, E, dt, model, fel, want_dt_next)

    def run_electrons(self, P, E, nsteps, dt, model=0, fel=0.5):
        return grmhd_run_electrons(self.ctx, P, E, nsteps, dt, model, fel)

    def divb(self, P):
        return grmhd_divb(self.ctx, P)

    def step_failures(self):
        return grmhd_step_failures(self.ctx)

    def set_tiles(self, which, tx, ty):
        grmhd_set_tiles(self.ctx, which, tx, ty)

    def get_tiles(self, which):
        return grmhd_get_tiles(self.ctx, which)
