"""ctypes binding of the DUWP CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  The product path (the HIP library and its Python binding) never
does.  The oracle is built from ``duwp_oracle.c`` with gcc by :func:`build`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "duwp_oracle.c")
LIB = os.path.join(HERE, "libduwp_oracle.so")

CLASSIFY, RESAMPLE, COLLIDE, STREAM, WAVE = 1, 2, 4, 8, 16
ALL = 0x1F


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, FP64, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


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
        ("flux_order", C.c_int32), ("absorb_stream", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        u32p = C.POINTER(C.c_uint32)
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Case), C.c_uint64, C.c_int32]
        L.orc_destroy.argtypes = [P]
        L.orc_num_particles.restype = C.c_int64
        L.orc_num_particles.argtypes = [P]
        L.orc_num_cells.restype = C.c_int32
        L.orc_num_cells.argtypes = [P]
        L.orc_get_step.restype = C.c_uint32
        L.orc_get_step.argtypes = [P]
        L.orc_get_state.argtypes = [P, dp, dp, dp, dp, i64p, dp, dp]
        L.orc_set_state.argtypes = [P, C.c_int64, dp, dp, dp, dp, i64p, dp, dp, C.c_uint32]
        L.orc_step.argtypes = [P, C.c_int32]
        L.orc_step_masked.argtypes = [P, C.c_int32]
        L.orc_get_diag.argtypes = [P, i32p, i32p, i32p, i32p, i64p, i64p]
        L.orc_get_cells.argtypes = [P, dp, dp, dp]
        L.orc_get_average.argtypes = [P, dp, i64p]
        L.orc_reset_average.argtypes = [P]
        L.orc_stress_heat.restype = C.c_int
        L.orc_stress_heat.argtypes = [P, dp]
        L.orc_philox.argtypes = [u32p, u32p, u32p]
        L.orc_eps.restype = C.c_double
        L.orc_eps.argtypes = [C.c_int32, C.c_double]
        L.orc_kfvs_half.argtypes = [dp, C.c_double, C.c_int32, dp]
        L.orc_wave_flux.argtypes = [P, dp, dp, dp]
        L.orc_scatter_pair.argtypes = [dp, dp, C.c_double, C.c_double, dp, dp]
        L.orc_constants.argtypes = [P, dp]
        _lib = L
    return _lib


def _p(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


def make_case(case) -> _Case:
    d = case.to_dict() if hasattr(case, "to_dict") else dict(case)
    c = _Case()
    for name, _ in _Case._fields_:
        setattr(c, name, d.get(name, 0))
    return c


def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    ctr = np.asarray(ctr, np.uint32)
    key = np.asarray(key, np.uint32)
    lib().orc_philox(_p(ctr, C.c_uint32), _p(key, C.c_uint32), _p(out, C.c_uint32))
    return out


def eps(law: int, x: float) -> float:
    return lib().orc_eps(law, x)


def kfvs_half(W, R, sign):
    W = np.asarray(W, np.float64)
    H = np.zeros(5)
    lib().orc_kfvs_half(_p(W), R, sign, _p(H))
    return H


def scatter_pair(xi_i, xi_j, u3, u4):
    a = np.asarray(xi_i, np.float64)
    b = np.asarray(xi_j, np.float64)
    oi = np.zeros(3)
    oj = np.zeros(3)
    lib().orc_scatter_pair(_p(a), _p(b), u3, u4, _p(oi), _p(oj))
    return oi, oj


class Oracle:
    """One case evolved by the plain CPU implementation."""

    def __init__(self, case, seed: int = 1, case_id: int = 0):
        self._c = make_case(case)
        self.case = case
        self.ptr = lib().orc_create(C.byref(self._c), seed, case_id)
        if not self.ptr:
            raise ValueError("oracle rejected the case description")
        self.ncells = case.ncells

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().orc_destroy(self.ptr)
            self.ptr = None

    @property
    def n(self) -> int:
        return lib().orc_num_particles(self.ptr)

    @property
    def step_index(self) -> int:
        return lib().orc_get_step(self.ptr)

    def step(self, nsteps: int = 1) -> None:
        if lib().orc_step(self.ptr, nsteps) != 0:
            raise RuntimeError("oracle step reported an error")

    def step_masked(self, mask: int) -> None:
        if lib().orc_step_masked(self.ptr, mask) != 0:
            raise RuntimeError("oracle step reported an error")

    def constants(self) -> dict:
        o = np.zeros(6)
        lib().orc_constants(self.ptr, _p(o))
        return dict(zip(["dx", "beta", "mu_ref", "upsilon", "c_ref", "coll_k"], o))

    def get_state(self) -> dict:
        n, Cn = self.n, self.ncells
        x, u, v, w = (np.zeros(n) for _ in range(4))
        off = np.zeros(Cn + 1, np.int64)
        psi_w = np.zeros(Cn * 5)
        cr = np.zeros(Cn)
        lib().orc_get_state(self.ptr, _p(x), _p(u), _p(v), _p(w), _p(off, C.c_int64), _p(psi_w), _p(cr))
        return dict(x=x, u=u, v=v, w=w, off=off, psi_w=psi_w.reshape(Cn, 5), cr_max=cr,
                    step=self.step_index)

    def set_state(self, st: dict) -> None:
        x = np.ascontiguousarray(st["x"], np.float64)
        u = np.ascontiguousarray(st["u"], np.float64)
        v = np.ascontiguousarray(st["v"], np.float64)
        w = np.ascontiguousarray(st["w"], np.float64)
        off = np.ascontiguousarray(st["off"], np.int64)
        psi = np.ascontiguousarray(st["psi_w"], np.float64).reshape(-1)
        cr = np.ascontiguousarray(st["cr_max"], np.float64)
        rc = lib().orc_set_state(self.ptr, len(x), _p(x), _p(u), _p(v), _p(w), _p(off, C.c_int64),
                                 _p(psi), _p(cr), int(st["step"]))
        if rc != 0:
            raise ValueError("oracle rejected the state")

    def diag(self) -> dict:
        Cn = self.ncells
        a, b, c, d = (np.zeros(Cn, np.int32) for _ in range(4))
        inj = np.zeros(2, np.int64)
        out = np.zeros(1, np.int64)
        lib().orc_get_diag(self.ptr, _p(a, C.c_int32), _p(b, C.c_int32), _p(c, C.c_int32),
                           _p(d, C.c_int32), _p(inj, C.c_int64), _p(out, C.c_int64))
        return dict(n_abs=a, n_new=b, n_cand=c, n_coll=d, n_inj=inj, n_out=int(out[0]))

    def cells(self) -> dict:
        Cn = self.ncells
        prim = np.zeros(Cn * 5)
        pt = np.zeros(Cn * 5)
        pp = np.zeros(Cn * 5)
        lib().orc_get_cells(self.ptr, _p(prim), _p(pt), _p(pp))
        return dict(prim=prim.reshape(Cn, 5), psi_t=pt.reshape(Cn, 5), psi_p=pp.reshape(Cn, 5))

    def stress_heat(self) -> np.ndarray:
        """(Pi, Q, Pi_p, Q_p, rho_w/rho_t) per cell of the current state, shape (C, 5)."""
        out = np.zeros((self.ncells, 5))
        if lib().orc_stress_heat(self.ptr, _p(out)) != 0:
            raise MemoryError("orc_stress_heat")
        return out

    def average(self):
        s = np.zeros(self.ncells * 5)
        cnt = np.zeros(1, np.int64)
        lib().orc_get_average(self.ptr, _p(s), _p(cnt, C.c_int64))
        return s.reshape(self.ncells, 5), int(cnt[0])

    def reset_average(self) -> None:
        lib().orc_reset_average(self.ptr)

    def wave_flux(self, Wl, Wr):
        a = np.asarray(Wl, np.float64)
        b = np.asarray(Wr, np.float64)
        F = np.zeros(5)
        lib().orc_wave_flux(self.ptr, _p(a), _p(b), _p(F))
        return F


def prim_from_psi(psi, R):
    """(rho,U,V,W,T) from conserved sums (rows of 5)."""
    psi = np.asarray(psi, np.float64)
    rho = psi[..., 0]
    with np.errstate(divide="ignore", invalid="ignore"):
        U = psi[..., 1] / rho
        V = psi[..., 2] / rho
        W = psi[..., 3] / rho
        T = (2.0 / (3.0 * R)) * (psi[..., 4] / rho - 0.5 * (U * U + V * V + W * W))
    return np.stack([rho, U, V, W, T], axis=-1)
