"""Ctypes binding of the plain FP64 CPU oracle (``qmc_oracle.c``).

TEST INFRASTRUCTURE.  Only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg import this package.  It never imports the GPU package and
the GPU package never imports it; the only shared code is ``qmc_inputs``,
which builds seeded inputs and does none of the method's arithmetic.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SPO_SPLINE, SPO_PLANEWAVE = 0, 1
J_NONE, J_PADE, J_BSPLINE = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, OpenMP over walkers)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        dp, ip, u8p, u32p = (C.POINTER(C.c_double), C.POINTER(C.c_int32),
                             C.POINTER(C.c_uint8), C.POINTER(C.c_uint32))
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_uniform2.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, dp]
        L.orc_gauss3.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, dp]
        L.orc_accept_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.orc_accept_uniform.restype = C.c_double
        L.orc_branch_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32]
        L.orc_branch_uniform.restype = C.c_double
        L.orc_dmc_run.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int,
                                  dp, dp, ip, ip, dp, dp, ip, C.c_int]
        L.orc_dmc_run.restype = C.c_int
        L.orc_init_position.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_double, dp]
        L.orc_spo_vgl.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_radial.argtypes = [C.c_void_p, C.c_int, C.c_double, dp]
        L.orc_inverse.argtypes = [C.c_int, dp, dp, dp, ip]
        L.orc_inverse.restype = C.c_int
        L.orc_sherman_morrison.argtypes = [C.c_int, dp, C.c_int, dp, C.c_double]
        L.orc_woodbury.argtypes = [C.c_int, dp, dp, C.c_int, ip, dp]
        L.orc_woodbury.restype = C.c_int
        L.orc_ewald.argtypes = [C.c_int, dp, dp, C.c_double, C.c_double]
        L.orc_ewald.restype = C.c_double
        L.orc_local_energy.argtypes = [C.c_void_p, dp, dp]
        L.orc_local_energy.restype = C.c_int
        L.orc_log_psi.argtypes = [C.c_void_p, dp, ip]
        L.orc_log_psi.restype = C.c_double
        L.orc_vmc_run.argtypes = [C.c_void_p, C.c_int, ip, dp, C.c_int, C.c_int, C.c_int, dp, u8p,
                                  dp, dp, dp, ip, dp, C.c_int]
        L.orc_vmc_run.restype = C.c_int
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


class _Sys(C.Structure):
    _fields_ = [
        ("n_up", C.c_int32), ("n_dn", C.c_int32), ("L", C.c_double),
        ("spo_kind", C.c_int32), ("n_orb", C.c_int32),
        ("gx", C.c_int32), ("gy", C.c_int32), ("gz", C.c_int32),
        ("coefs", C.POINTER(C.c_double)), ("pw_k", C.POINTER(C.c_double)),
        ("pw_kind", C.POINTER(C.c_int32)),
        ("n_ions", C.c_int32), ("ion_pos", C.POINTER(C.c_double)), ("ion_Z", C.POINTER(C.c_double)),
        ("j2_kind", C.c_int32), ("j2_a", C.c_double), ("j2_b", C.c_double),
        ("j2_M", C.c_int32), ("j2_rc", C.c_double), ("j2_p", C.POINTER(C.c_double)),
        ("j2_cusp_same", C.c_double), ("j2_cusp_opp", C.c_double),
        ("j1_kind", C.c_int32), ("j1_M", C.c_int32), ("j1_rc", C.c_double),
        ("j1_p", C.POINTER(C.c_double)), ("j1_cusp", C.c_double),
        ("sigma", C.c_double), ("seed", C.c_uint64),
        ("coulomb", C.c_int32), ("ewald_kappa", C.c_double), ("all_electron", C.c_int32),
        ("j3_mei", C.c_int32), ("j3_mee", C.c_int32), ("j3_rc", C.c_double),
        ("j3_gamma", C.POINTER(C.c_double)),
    ]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class OracleSystem:
    """A workload translated into the oracle's system struct (arrays kept alive here)."""

    def __init__(self, wl, spo: str = "spline", kappa: float = 0.0, coulomb=None):
        self.wl = wl
        keep = []

        def arr(x, dt=np.float64):
            a = np.ascontiguousarray(np.asarray(x, dtype=dt))
            keep.append(a)
            return a

        s = _Sys()
        s.n_up, s.n_dn, s.L = wl.n_up, wl.n_dn, wl.L
        s.n_orb = wl.n_orb
        if spo == "spline":
            s.spo_kind = SPO_SPLINE
            s.gx, s.gy, s.gz = wl.grid
            s.coefs = _dp(arr(wl.coefs))
        else:
            s.spo_kind = SPO_PLANEWAVE
            s.pw_k = _dp(arr(wl.pw_k))
            s.pw_kind = _ip(arr(wl.pw_kind, np.int32))
        s.n_ions = wl.n_ions
        s.ion_pos = _dp(arr(wl.ion_pos.reshape(-1, 3) if wl.n_ions else np.zeros((1, 3))))
        s.ion_Z = _dp(arr(wl.ion_Z if wl.n_ions else np.zeros(1)))
        j2 = wl.j2
        if j2 is None:
            s.j2_kind = J_NONE
        elif j2["kind"] == "pade":
            s.j2_kind, s.j2_a, s.j2_b = J_PADE, j2["a"], j2["b"]
        else:
            s.j2_kind, s.j2_M, s.j2_rc = J_BSPLINE, j2["M"], j2["rc"]
            s.j2_p = _dp(arr(j2["p"]))
            s.j2_cusp_same, s.j2_cusp_opp = j2["cusp_same"], j2["cusp_opp"]
        j1 = wl.j1
        if j1 is None or wl.n_ions == 0:
            s.j1_kind = J_NONE
        else:
            s.j1_kind, s.j1_M, s.j1_rc = J_BSPLINE, j1["M"], j1["rc"]
            s.j1_p = _dp(arr(j1["p"]))
            s.j1_cusp = j1["cusp"]
        s.sigma, s.seed = wl.sigma, wl.seed
        s.coulomb = int((wl.hamiltonian == "coulomb") if coulomb is None else coulomb)
        s.ewald_kappa = kappa
        ae = bool(getattr(wl, "all_electron", False))
        drift = bool(getattr(wl, "drift", False))
        s.all_electron = (2 if drift else 1) if ae else (3 if drift else 0)
        j3 = getattr(wl, "j3", None)
        if j3 is not None and wl.n_ions > 0:
            s.j3_mei, s.j3_mee, s.j3_rc = j3["m_ei"], j3["m_ee"], j3["rc"]
            s.j3_gamma = _dp(arr(j3["gamma"]))
        self.s = s
        self._keep = keep

    @property
    def ptr(self):
        return C.byref(self.s)

    # -- single-function entry points used by the pins -------------------------------
    def spo_vgl(self, r):
        n = self.wl.n_orb
        v, g, l = np.zeros(n), np.zeros(3 * n), np.zeros(n)
        r = np.ascontiguousarray(r, dtype=np.float64)
        lib().orc_spo_vgl(self.ptr, _dp(r), _dp(v), _dp(g), _dp(l))
        return v, g.reshape(3, n), l

    def radial(self, kind: int, r: float):
        out = np.zeros(3)
        lib().orc_radial(self.ptr, kind, float(r), _dp(out))
        return out

    def local_energy(self, pos):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        out = np.zeros(4)
        bad = lib().orc_local_energy(self.ptr, _dp(pos), _dp(out))
        if bad:
            raise ValueError("singular Slater matrix")
        return out

    def log_psi(self, pos):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        sg = np.zeros(1, dtype=np.int32)
        lp = lib().orc_log_psi(self.ptr, _dp(pos), _ip(sg))
        return lp, int(sg[0])

    def run(self, walker_ids, n_sweeps: int, measure_every: int = 1, sweep0: int = 0,
            init_pos=None, trace: bool = False, bits: bool = True, threads: int = 0):
        """Run the chains of ``walker_ids`` for ``n_sweeps`` sweeps; returns a dict of arrays."""
        wl = self.wl
        N = wl.n_elec
        ids = np.ascontiguousarray(np.asarray(walker_ids, dtype=np.int32))
        W = len(ids)
        n_meas = n_sweeps // measure_every if measure_every > 0 else 0
        E = np.zeros((W, max(n_meas, 1), 4))
        acc = np.zeros((W, n_sweeps, N), dtype=np.uint8) if bits else None
        tr = np.zeros((W, n_sweeps, N, 3)) if trace else None
        fp = np.zeros((W, N, 3))
        ld = np.zeros((W, 2))
        sg = np.zeros((W, 2), dtype=np.int32)
        ldlu = np.zeros((W, 2))
        ip = None
        if init_pos is not None:
            ip = np.ascontiguousarray(np.asarray(init_pos, dtype=np.float64).reshape(W, N, 3))
        rc = lib().orc_vmc_run(
            self.ptr, W, _ip(ids), _dp(ip) if ip is not None else None, sweep0, n_sweeps,
            measure_every, _dp(E), acc.ctypes.data_as(C.POINTER(C.c_uint8)) if bits else None,
            _dp(tr) if trace else None, _dp(fp), _dp(ld), _ip(sg), _dp(ldlu), threads)
        if rc:
            raise ValueError(f"singular Slater matrix at initialisation of walker {ids[rc - 1]}")
        return {"energies": E[:, :n_meas], "accept": acc, "trace": tr, "final_pos": fp,
                "logdet": ld, "sign": sg, "logdet_lu": ldlu}


    def dmc(self, n_slots: int, n_target: int, n_steps: int, e_trial: float = float("nan"),
            feedback: float = 1.0, sweep0: int = 0, threads: int = 0):
        """Diffusion Monte Carlo on ``n_slots`` walker slots (the first ``n_target`` alive at
        the start, drawn from the INIT stream with walker id = slot): per-step statistics
        (E, sum of weights, population, E_T used, dropped copies, node-crossing moves rejected),
        per-slot weights,
        multiplicities, copy plans and local energies, final positions and signs."""
        N = self.wl.n_elec
        st = np.zeros((n_steps, 6))
        w = np.zeros((n_steps, n_slots))
        m = np.zeros((n_steps, n_slots), dtype=np.int32)
        pl = np.zeros((n_steps, n_slots), dtype=np.int32)
        en = np.zeros((n_steps, n_slots))
        fp = np.zeros((n_slots, N, 3))
        fs = np.zeros(n_slots, dtype=np.int32)
        rc = lib().orc_dmc_run(self.ptr, n_slots, n_target, e_trial, feedback, sweep0, n_steps, _dp(st),
                               _dp(w), _ip(m), _ip(pl), _dp(en), _dp(fp), _ip(fs), threads)
        if rc == -2:
            raise ValueError("DMC needs drift-diffusion moves (drift)")
        if rc == -1:
            raise ValueError("the population died out")
        if rc:
            raise ValueError(f"singular Slater matrix at initialisation of slot {rc - 1}")
        return {"stats": st, "weights": w, "mult": m, "plan": pl, "energies": en,
                "final_pos": fp, "final_sign": fs}


# -- free functions ------------------------------------------------------------------

def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    p = C.POINTER(C.c_uint32)
    lib().orc_philox4x32_10(c.ctypes.data_as(p), k.ctypes.data_as(p), o.ctypes.data_as(p))
    return o


def uniform2(seed, purpose, sub, walker, sweep, electron):
    u = np.zeros(2)
    lib().orc_uniform2(seed, purpose, sub, walker, sweep, electron, _dp(u))
    return u


def gauss3(seed, walker, sweep, electron):
    xi = np.zeros(3)
    lib().orc_gauss3(seed, walker, sweep, electron, _dp(xi))
    return xi


def accept_uniform(seed, walker, sweep, electron):
    return lib().orc_accept_uniform(seed, walker, sweep, electron)


def branch_uniform(seed, slot, step):
    return lib().orc_branch_uniform(seed, slot, step)


def init_position(seed, walker, electron, L):
    r = np.zeros(3)
    lib().orc_init_position(seed, walker, electron, L, _dp(r))
    return r


def inverse(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    B = np.zeros_like(A)
    la = np.zeros(1)
    sg = np.zeros(1, dtype=np.int32)
    bad = lib().orc_inverse(n, _dp(A), _dp(B), _dp(la), _ip(sg))
    if bad:
        raise ValueError("singular matrix")
    return B, float(la[0]), int(sg[0])


def sherman_morrison(B, k, v, R):
    B = np.ascontiguousarray(B, dtype=np.float64).copy()
    v = np.ascontiguousarray(v, dtype=np.float64)
    lib().orc_sherman_morrison(B.shape[0], _dp(B), int(k), _dp(v), float(R))
    return B


def woodbury(A, B, rows, V):
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64).copy()
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    V = np.ascontiguousarray(V, dtype=np.float64)
    bad = lib().orc_woodbury(A.shape[0], _dp(A), _dp(B), len(rows), _ip(rows), _dp(V))
    if bad:
        raise ValueError("singular capacitance matrix")
    return B


def ewald(pos, q, L, kappa=0.0):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    return lib().orc_ewald(len(q), _dp(pos), _dp(q), float(L), float(kappa))


def max_threads():
    return lib().orc_max_threads()
