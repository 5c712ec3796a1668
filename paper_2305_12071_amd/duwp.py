"""Python binding of libduwp (ctypes).  Argument marshalling only: every stage
of the DUWP step runs in the library's HIP kernels.

The library is built in-tree by ``paper_2305_12071_amd.build``; importing this
module does not build it, and :func:`lib` raises if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(PKG, "libduwp.so")

FP64, MIXED = 0, 1
M_PRIM, M_PSI_T, M_PSI_W, M_PSI_P, M_AVG_PRIM, M_AVG_SUM, M_STRESS_HEAT = range(7)

STATUS = {0: "ok", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ECAPACITY", -5: "ESTATE", -6: "ERANGE"}


class DuwpError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({_strerror(status)})")


class _Case(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("ncells", C.c_int32),
        ("x_lo", C.c_double), ("x_hi", C.c_double), ("x_split", C.c_double),
        ("rho_L", C.c_double), ("u_L", C.c_double), ("T_L", C.c_double),
        ("rho_R", C.c_double), ("u_R", C.c_double), ("T_R", C.c_double),
        ("R", C.c_double), ("omega", C.c_double), ("T_ref", C.c_double),
        ("m_mol", C.c_double), ("d_ref", C.c_double),
        ("lambda_ref", C.c_double), ("rho_ref", C.c_double),
        ("m_particle", C.c_double), ("dt", C.c_double),
        ("bc_lo", C.c_int32), ("bc_hi", C.c_int32),
        ("classify_law", C.c_int32), ("eps_law", C.c_int32), ("dsmc_full_dt", C.c_int32),
        ("flux_order", C.c_int32), ("absorb_stream", C.c_int32), ("reserved_case", C.c_int32),
        ("capacity", C.c_int64),
    ]


TUNE_FIELDS = ("scatter_items", "big_block", "big_blocks_per_cu", "big_min_particles", "big_min_candidates",
               "collide_by_cell_max", "count_dests", "collide_blocks_per_cu")


class _Tune(C.Structure):
    _fields_ = [(f, C.c_int32) for f in TUNE_FIELDS]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class _Opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("precision", C.c_int32), ("use_graph", C.c_int32),
                ("stream", C.c_void_p), ("headroom", C.c_double), ("block_cells", C.c_int32),
                ("reserved", C.c_int32), ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", C.c_void_p),
                ("tune", _Tune)]


class _State(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("ncells", C.c_int32), ("step", C.c_uint32),
                ("x", C.POINTER(C.c_double)), ("u", C.POINTER(C.c_double)),
                ("v", C.POINTER(C.c_double)), ("w", C.POINTER(C.c_double)),
                ("off", C.POINTER(C.c_int64)), ("psi_w", C.POINTER(C.c_double)),
                ("cr_max", C.POINTER(C.c_double)), ("psi_p", C.POINTER(C.c_double)),
                ("avg_sum", C.POINTER(C.c_double)), ("avg_count", C.c_int64)]


class TorchAllocator:
    """torch's caching allocator as the library's device memory provider: the
    callbacks the context calls at duwp_init and duwp_destroy (kept alive here
    while the context lives)."""

    def __init__(self, stream=None):
        import torch
        self.torch = torch
        self.device = torch.cuda.current_device()
        self.stream = stream
        self.live = 0
        self.last_error = None

        def _alloc(nbytes, _ctx):
            try:
                ptr = self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception as e:   # out of memory: the library reports DUWP_ENOMEM
                self.last_error = f"{type(e).__name__} for {int(nbytes)} bytes: {e}"
                return None
            self.live += 1
            return ptr

        def _free(ptr, _ctx):
            self.torch.cuda.caching_allocator_delete(ptr)
            self.live -= 1

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


_lib = None
_live = None     # contexts not yet closed (closed at exit, while torch is still loaded)


def _close_all():
    for sim in list(_live or ()):
        try:
            sim.close()
        except Exception:
            pass


def lib():
    """Load libduwp.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: build it with `python -m paper_2305_12071_amd.build`")
        try:
            # torch ships its own HIP runtime with the same soname as ROCm's; loading it
            # first makes libduwp bind to that one, so the process holds a single HIP
            # runtime and torch's streams are valid handles for the library.
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        i32p = C.POINTER(C.c_int32)
        i64p = C.POINTER(C.c_int64)
        L.duwp_init.restype = C.c_int
        L.duwp_init.argtypes = [C.POINTER(P), C.POINTER(_Case), C.c_int32, C.POINTER(_Opts)]
        L.duwp_step.restype = C.c_int
        L.duwp_step.argtypes = [P, C.c_int32]
        L.duwp_moments.restype = C.c_int
        L.duwp_moments.argtypes = [P, C.c_int32, C.c_int32, dp, C.c_int64, C.c_int32]
        L.duwp_moments_noalloc.restype = C.c_int
        L.duwp_moments_noalloc.argtypes = [P, C.c_int32, C.c_int32, C.c_void_p, C.c_int64]
        L.duwp_avg_count.restype = C.c_int64
        L.duwp_avg_count.argtypes = [P]
        L.duwp_reset_average.restype = C.c_int
        L.duwp_reset_average.argtypes = [P]
        L.duwp_counts.restype = C.c_int
        L.duwp_counts.argtypes = [P, C.c_int32, i64p, i32p, C.POINTER(C.c_uint32)]
        L.duwp_diag.restype = C.c_int
        L.duwp_diag.argtypes = [P, C.c_int32, i32p, i32p, i32p, i32p, i64p, i64p]
        L.duwp_get_state.restype = C.c_int
        L.duwp_get_state.argtypes = [P, C.c_int32, C.POINTER(_State)]
        L.duwp_set_state.restype = C.c_int
        L.duwp_set_state.argtypes = [P, C.c_int32, C.POINTER(_State)]
        L.duwp_profile.restype = C.c_int
        L.duwp_profile.argtypes = [P, C.c_int32, C.POINTER(C.c_char_p), dp, C.c_int32, i32p]
        L.duwp_particle_steps.restype = C.c_int
        L.duwp_particle_steps.argtypes = [P, i64p, C.c_int32]
        L.duwp_sync.restype = C.c_int
        L.duwp_sync.argtypes = [P]
        L.duwp_destroy.restype = None
        L.duwp_destroy.argtypes = [P]
        L.duwp_strerror.restype = C.c_char_p
        L.duwp_strerror.argtypes = [C.c_int]
        _lib = L
    return _lib


def hip_runtimes_loaded():
    """Paths of the HIP runtime libraries mapped into this process."""
    import re
    with open("/proc/self/maps") as f:
        maps = f.read()
    return sorted(set(re.findall(r"(/\S*libamdhip64\S*)", maps)))


def _strerror(s: int) -> str:
    try:
        return lib().duwp_strerror(s).decode()
    except Exception:  # pragma: no cover - library missing
        return "?"


def _check(s: int, what: str) -> None:
    if s != 0:
        raise DuwpError(s, what)


def _p(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


def make_case(case) -> _Case:
    d = case.to_dict() if hasattr(case, "to_dict") else dict(case)
    c = _Case()
    for name, _ in _Case._fields_:
        setattr(c, name, d.get(name, 0))
    return c


def _torch_gpu() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def current_stream():
    """hipStream_t of torch's current stream (torch is only plumbing here), or None."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


class Sim:
    """A set of independent cases advanced together by the HIP pipeline."""

    def __init__(self, cases, seed: int = 1, precision: int = FP64, use_graph: bool = False,
                 stream=None, headroom: float = 0.0, block_cells: int = 0, tune: dict | None = None,
                 allocator: str = "torch"):
        """allocator: "torch" (device buffers from torch's caching allocator, the
        default when torch sees a GPU) or "hip" (the library's hipMalloc)."""
        if not isinstance(cases, (list, tuple)):
            cases = [cases]
        self.cases = list(cases)
        arr = (_Case * len(cases))(*[make_case(c) for c in cases])
        self._arr = arr
        o = _Opts()
        o.seed = seed
        o.precision = precision
        o.use_graph = 1 if use_graph else 0
        s = current_stream() if stream is None else stream
        o.stream = C.c_void_p(s) if s else None
        o.headroom = headroom
        o.block_cells = block_cells
        for k, v in (tune or {}).items():
            if k not in TUNE_FIELDS:
                raise ValueError(f"unknown tuning field {k}")
            setattr(o.tune, k, int(v))
        self.allocator = None
        if allocator == "torch" and _torch_gpu():
            self.allocator = TorchAllocator()
            o.alloc, o.free = self.allocator.alloc, self.allocator.free
        elif allocator not in ("torch", "hip"):
            raise ValueError(f"allocator {allocator!r}")
        self.precision = precision
        self.ptr = C.c_void_p()
        st = lib().duwp_init(C.byref(self.ptr), arr, len(cases), C.byref(o))
        if st != 0 and self.allocator is not None and self.allocator.last_error:
            raise DuwpError(st, f"duwp_init (torch allocator: {self.allocator.last_error[:300]})")
        _check(st, "duwp_init")
        global _live
        if _live is None:
            import atexit
            import weakref
            _live = weakref.WeakSet()
            atexit.register(_close_all)
        _live.add(self)

    def close(self) -> None:
        if getattr(self, "ptr", None) and self.ptr.value:
            lib().duwp_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:       # interpreter shutdown: the library may be gone already
            pass

    def step(self, n: int = 1) -> None:
        _check(lib().duwp_step(self.ptr, n), "duwp_step")

    def counts(self, case_id: int = 0):
        n = C.c_int64()
        nc = C.c_int32()
        st = C.c_uint32()
        _check(lib().duwp_counts(self.ptr, case_id, C.byref(n), C.byref(nc), C.byref(st)), "duwp_counts")
        return n.value, nc.value, st.value

    def n_particles(self, case_id: int = 0) -> int:
        return self.counts(case_id)[0]

    def total_particles(self) -> int:
        return sum(self.n_particles(k) for k in range(len(self.cases)))

    @property
    def step_index(self) -> int:
        return self.counts(0)[2]

    def moments(self, case_id: int = 0, what: int = M_PRIM) -> np.ndarray:
        nc = self.cases[case_id].ncells
        out = np.zeros(nc * 5)
        _check(lib().duwp_moments(self.ptr, case_id, what, _p(out), out.size, 0), "duwp_moments")
        return out.reshape(nc, 5)

    def moments_noalloc(self, out_ptr: int, length: int, case_id: int = 0, what: int = M_PRIM) -> None:
        """duwp_moments_noalloc into device memory at out_ptr (length doubles), queued
        on the context's stream; nothing is allocated and nothing waits."""
        _check(lib().duwp_moments_noalloc(self.ptr, case_id, what, C.c_void_p(out_ptr), length),
               "duwp_moments_noalloc")

    def avg_count(self) -> int:
        return lib().duwp_avg_count(self.ptr)

    def reset_average(self) -> None:
        _check(lib().duwp_reset_average(self.ptr), "duwp_reset_average")

    def average(self, case_id: int = 0):
        return self.moments(case_id, M_AVG_SUM), self.avg_count()

    def diag(self, case_id: int = 0) -> dict:
        nc = self.cases[case_id].ncells
        a, b, c, d = (np.zeros(nc, np.int32) for _ in range(4))
        inj = np.zeros(2, np.int64)
        out = np.zeros(1, np.int64)
        _check(lib().duwp_diag(self.ptr, case_id, _p(a, C.c_int32), _p(b, C.c_int32), _p(c, C.c_int32),
                               _p(d, C.c_int32), _p(inj, C.c_int64), _p(out, C.c_int64)), "duwp_diag")
        return dict(n_abs=a, n_new=b, n_cand=c, n_coll=d, n_inj=inj, n_out=int(out[0]))

    def get_state(self, case_id: int = 0) -> dict:
        n, nc, step = self.counts(case_id)
        x, u, v, w = (np.zeros(n) for _ in range(4))
        off = np.zeros(nc + 1, np.int64)
        psi = np.zeros(nc * 5)
        cr = np.zeros(nc)
        pp = np.zeros(nc * 5)
        av = np.zeros(nc * 5)
        s = _State(n, nc, step, _p(x), _p(u), _p(v), _p(w), _p(off, C.c_int64), _p(psi), _p(cr), _p(pp),
                   _p(av), 0)
        _check(lib().duwp_get_state(self.ptr, case_id, C.byref(s)), "duwp_get_state")
        return dict(x=x, u=u, v=v, w=w, off=off, psi_w=psi.reshape(nc, 5), cr_max=cr, step=s.step,
                    psi_p=pp.reshape(nc, 5), avg_sum=av.reshape(nc, 5), avg_count=int(s.avg_count),
                    precision=self.precision)

    def set_state(self, st: dict, case_id: int = 0) -> None:
        x = np.ascontiguousarray(st["x"], np.float64)
        u = np.ascontiguousarray(st["u"], np.float64)
        v = np.ascontiguousarray(st["v"], np.float64)
        w = np.ascontiguousarray(st["w"], np.float64)
        off = np.ascontiguousarray(st["off"], np.int64)
        psi = np.ascontiguousarray(st["psi_w"], np.float64).reshape(-1)
        cr = np.ascontiguousarray(st["cr_max"], np.float64)
        # particle moments travel with the state when it has them (a resume bit for
        # bit); without them the library sums them from the particles.  A state
        # that the other precision saved leaves them behind (the load rounds its
        # particles); drop "psi_p" from one whose particles were edited.
        pp = st.get("psi_p")
        if st.get("precision", self.precision) != self.precision:
            pp = None
        pp = None if pp is None else np.ascontiguousarray(pp, np.float64).reshape(-1)
        # the running time average travels with a checkpoint that has it
        av = st.get("avg_sum")
        av = None if av is None else np.ascontiguousarray(av, np.float64).reshape(-1)
        s = _State(len(x), len(off) - 1, int(st["step"]), _p(x), _p(u), _p(v), _p(w),
                   _p(off, C.c_int64), _p(psi), _p(cr), None if pp is None else _p(pp),
                   None if av is None else _p(av), int(st.get("avg_count", 0)) if av is not None else 0)
        _check(lib().duwp_set_state(self.ptr, case_id, C.byref(s)), "duwp_set_state")

    def profile(self, nsteps: int = 3) -> dict:
        cap = 32
        names = (C.c_char_p * cap)()
        ms = np.zeros(cap)
        cnt = C.c_int32()
        _check(lib().duwp_profile(self.ptr, nsteps, names, _p(ms), cap, C.byref(cnt)), "duwp_profile")
        return {names[i].decode(): float(ms[i]) for i in range(cnt.value)}

    def particle_steps(self, reset: bool = False) -> int:
        v = C.c_int64()
        _check(lib().duwp_particle_steps(self.ptr, C.byref(v), 1 if reset else 0), "duwp_particle_steps")
        return v.value

    def sync(self) -> None:
        _check(lib().duwp_sync(self.ptr), "duwp_sync")
