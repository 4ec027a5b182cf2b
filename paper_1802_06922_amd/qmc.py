"""Thin ctypes binding of ``libqmc.so`` (the C ABI declared in ``include/qmc.h``).

Argument marshalling only: every step of the VMC path runs in the library's
HIP kernels.  PyTorch supplies the HIP stream and, optionally, the device
memory arena.  Importing this module does not need a GPU; creating a
``System`` does, and fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libqmc.so")

QMC_OK, QMC_ERR_ARG, QMC_ERR_OOM, QMC_ERR_SINGULAR, QMC_ERR_DEVICE, QMC_ERR_STATE, QMC_ERR_NUMERIC = range(7)
QMC_FP64, QMC_MIXED = 0, 1
QMC_J_NONE, QMC_J_PADE, QMC_J_BSPLINE = 0, 1, 2
QMC_H_KINETIC, QMC_H_COULOMB_EWALD = 0, 1
KERNEL_GATHER, KERNEL_CHAIN, KERNEL_MEASURE, KERNEL_REBUILD = 0, 1, 2, 3

EXPORTS = [
    "qmc_create_system", "qmc_load_spline_table", "qmc_init_walkers", "qmc_sweep",
    "qmc_measure_local_energy", "qmc_get_walkers", "qmc_get_accept_log", "qmc_get_counters", "qmc_recompute",
    "qmc_eval_spo_vgl", "qmc_set_timing", "qmc_kernel_timing", "qmc_destroy_system",
    "qmc_last_error", "qmc_estimate_device_bytes", "qmc_set_delay_rank", "qmc_autotune_delay",
    "qmc_get_last_energies", "qmc_batch_create", "qmc_batch_sweep", "qmc_batch_set_graph",
    "qmc_batch_timing", "qmc_batch_destroy", "qmc_max_delay_rank", "qmc_autotune_gather",
    "qmc_set_gather_lanes", "qmc_run_steps", "qmc_dmc_init", "qmc_dmc_steps", "qmc_dmc_get", "qmc_dmc_get_branching",
    "qmc_get_precision_stats", "qmc_eval_spo_vgl_noalloc", "qmc_set_sweep_index",
]
NOALLOC_DOUBLES = 1 << 19   # QMC_NOALLOC_DOUBLES


class QMCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qmc status {status}: {msg}")
        self.status = status


class Desc(C.Structure):
    _fields_ = [
        ("n_up", C.c_int32), ("n_dn", C.c_int32), ("L", C.c_double),
        ("n_ions", C.c_int32), ("ion_pos", C.POINTER(C.c_double)), ("ion_Z", C.POINTER(C.c_double)),
        ("precision", C.c_int32), ("delay_rank", C.c_int32), ("recompute_period", C.c_int32),
        ("sigma", C.c_double), ("seed", C.c_uint64), ("hamiltonian", C.c_int32),
        ("j2_kind", C.c_int32), ("j2_params", C.POINTER(C.c_double)), ("j2_n", C.c_int32),
        ("j2_rcut", C.c_double), ("j2_cusp_same", C.c_double), ("j2_cusp_opp", C.c_double),
        ("j1_kind", C.c_int32), ("j1_params", C.POINTER(C.c_double)), ("j1_n", C.c_int32),
        ("j1_rcut", C.c_double), ("j1_cusp", C.c_double), ("tie_guard", C.c_double),
        ("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("move_kind", C.c_int32),
        ("j3_m_ei", C.c_int32), ("j3_m_ee", C.c_int32), ("j3_rcut", C.c_double),
        ("j3_gamma", C.POINTER(C.c_double)),
    ]


_lib = None


def load_library():
    """Load libqmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch's HIP runtime must be the one the library binds to (one runtime per process),
    # so torch is loaded before the library.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python paper_1802_06922_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, dp, st = C.c_void_p, C.POINTER(C.c_double), C.c_int
    L.qmc_create_system.argtypes = [C.POINTER(Desc), vp, C.POINTER(vp)]
    L.qmc_load_spline_table.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, C.c_int32, C.c_int32]
    L.qmc_init_walkers.argtypes = [vp, C.c_int32, dp]
    L.qmc_sweep.argtypes = [vp, C.c_int32, C.POINTER(C.c_uint64)]
    L.qmc_measure_local_energy.argtypes = [vp, vp, C.c_int32]
    L.qmc_get_walkers.argtypes = [vp, dp, dp, C.POINTER(C.c_int32)]
    L.qmc_get_accept_log.argtypes = [vp, C.POINTER(C.c_uint8)]
    L.qmc_get_counters.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    L.qmc_recompute.argtypes = [vp, dp]
    L.qmc_eval_spo_vgl.argtypes = [vp, C.c_int32, dp, dp]
    L.qmc_eval_spo_vgl_noalloc.argtypes = [vp, C.c_int32, dp, dp]
    L.qmc_set_sweep_index.argtypes = [vp, C.c_uint64]
    L.qmc_set_timing.argtypes = [vp, C.c_int32]
    L.qmc_kernel_timing.argtypes = [vp, C.c_int32, dp, C.POINTER(C.c_int64), C.c_int32]
    L.qmc_destroy_system.argtypes = [vp]
    L.qmc_last_error.argtypes = [vp]
    L.qmc_last_error.restype = C.c_char_p
    L.qmc_estimate_device_bytes.argtypes = [C.POINTER(Desc), C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    L.qmc_estimate_device_bytes.restype = C.c_size_t
    ip = C.POINTER(C.c_int32)
    L.qmc_set_delay_rank.argtypes = [vp, C.c_int32]
    L.qmc_autotune_delay.argtypes = [vp, ip, C.c_int32, C.c_int32, ip, dp]
    L.qmc_get_last_energies.argtypes = [vp, dp]
    L.qmc_batch_create.argtypes = [C.POINTER(vp), C.c_int32, vp, C.POINTER(vp)]
    L.qmc_batch_sweep.argtypes = [vp, C.c_int32, C.c_int32]
    L.qmc_batch_set_graph.argtypes = [vp, C.c_int32]
    L.qmc_batch_timing.argtypes = [vp, dp, C.POINTER(C.c_int64), C.c_int32]
    L.qmc_batch_destroy.argtypes = [vp]
    L.qmc_autotune_gather.argtypes = [vp, C.c_int32, ip, dp]
    L.qmc_set_gather_lanes.argtypes = [vp, C.c_int32]
    L.qmc_run_steps.argtypes = [vp, C.c_int32, vp]
    L.qmc_dmc_init.argtypes = [vp, C.c_int32, C.c_double, C.c_double]
    L.qmc_dmc_steps.argtypes = [vp, C.c_int32, vp]
    L.qmc_dmc_get.argtypes = [vp, dp, dp, dp, C.POINTER(C.c_int32)]
    L.qmc_dmc_get_branching.argtypes = [vp, dp, dp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.qmc_max_delay_rank.argtypes = [C.POINTER(Desc)]
    L.qmc_get_precision_stats.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                          C.POINTER(C.c_int32), ip]
    L.qmc_max_delay_rank.restype = C.c_int32
    for name in EXPORTS:
        if name not in ("qmc_last_error", "qmc_estimate_device_bytes", "qmc_max_delay_rank"):
            getattr(L, name).restype = st
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_desc(wl, keep: list, arena=None, arena_bytes: int = 0, tie_guard: float = 0.0) -> Desc:
    """Translate a ``qmc_inputs.Workload`` into the C descriptor (arrays appended to ``keep``)."""
    def arr(x):
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        keep.append(a)
        return a

    d = Desc()
    d.n_up, d.n_dn, d.L = wl.n_up, wl.n_dn, wl.L
    d.n_ions = wl.n_ions
    if wl.n_ions:
        d.ion_pos = _dp(arr(wl.ion_pos.reshape(-1)))
        d.ion_Z = _dp(arr(wl.ion_Z))
    d.precision = QMC_MIXED if wl.precision == "mixed" else QMC_FP64
    d.delay_rank = wl.delay_rank
    d.recompute_period = wl.recompute_period
    d.sigma, d.seed = wl.sigma, wl.seed
    d.hamiltonian = QMC_H_COULOMB_EWALD if wl.hamiltonian == "coulomb" else QMC_H_KINETIC
    j2 = wl.j2
    if j2 is None:
        d.j2_kind = QMC_J_NONE
    elif j2["kind"] == "pade":
        d.j2_kind = QMC_J_PADE
        d.j2_params = _dp(arr([j2["a"], j2["b"]]))
        d.j2_n = 2
    else:
        d.j2_kind = QMC_J_BSPLINE
        d.j2_params = _dp(arr(j2["p"]))
        d.j2_n = len(j2["p"])
        d.j2_rcut, d.j2_cusp_same, d.j2_cusp_opp = j2["rc"], j2["cusp_same"], j2["cusp_opp"]
    j1 = wl.j1
    if j1 is None or wl.n_ions == 0:
        d.j1_kind = QMC_J_NONE
    else:
        d.j1_kind = QMC_J_BSPLINE
        d.j1_params = _dp(arr(j1["p"]))
        d.j1_n = len(j1["p"])
        d.j1_rcut, d.j1_cusp = j1["rc"], j1["cusp"]
    d.tie_guard = tie_guard
    d.arena = arena
    d.arena_bytes = arena_bytes
    ae = bool(getattr(wl, "all_electron", False))
    drift = bool(getattr(wl, "drift", False))
    d.move_kind = (2 if drift else 1) if ae else (3 if drift else 0)
    j3 = getattr(wl, "j3", None)
    if j3 is not None and wl.n_ions > 0:
        d.j3_m_ei, d.j3_m_ee, d.j3_rcut = j3["m_ei"], j3["m_ee"], j3["rc"]
        d.j3_gamma = _dp(arr(j3["gamma"]))
    return d


class System:
    """One VMC system on the current GPU: a handle of the C library."""

    def __init__(self, wl, n_walkers: Optional[int] = None, init: bool = True, stream=None,
                 use_torch_arena: bool = False, tie_guard: float = 0.0, init_pos=None):
        import torch
        self.L = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("the QMC library needs a ROCm GPU")
        self.wl = wl
        self.W = int(n_walkers if n_walkers is not None else wl.n_walkers)
        self._keep: list = []
        self._arena = None
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        arena_ptr, arena_bytes = None, 0
        desc = make_desc(wl, self._keep, tie_guard=tie_guard)
        if use_torch_arena:
            g = wl.grid
            nbytes = self.L.qmc_estimate_device_bytes(C.byref(desc), self.W, g[0], g[1], g[2])
            if nbytes == 0:
                raise QMCError(QMC_ERR_ARG, "qmc_estimate_device_bytes rejected the descriptor")
            self._arena = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            arena_ptr, arena_bytes = self._arena.data_ptr(), nbytes
            desc.arena, desc.arena_bytes = arena_ptr, arena_bytes
        h = C.c_void_p()
        self._check(self.L.qmc_create_system(C.byref(desc), C.c_void_p(stream.cuda_stream), C.byref(h)), None)
        self.h = h
        coefs = np.ascontiguousarray(wl.coefs)
        dtype = 8 if coefs.dtype == np.float64 else 4
        if coefs.dtype not in (np.float64, np.float32):
            raise TypeError("coefs must be float64 or float32")
        g = wl.grid
        self._check(self.L.qmc_load_spline_table(h, g[0], g[1], g[2], wl.n_orb,
                                                 coefs.ctypes.data_as(C.c_void_p), dtype, 0))
        if init:
            self.init_walkers(self.W, init_pos)

    # -- plumbing ---------------------------------------------------------------------
    def _check(self, status: int, h="self"):
        if status != QMC_OK:
            handle = self.h if h == "self" else None
            msg = self.L.qmc_last_error(handle)
            raise QMCError(status, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.L.qmc_destroy_system(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C ABI calls ----------------------------------------------------------------------
    def init_walkers(self, n_walkers: int, pos=None):
        self.W = int(n_walkers)
        p = None
        if pos is not None:
            pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(self.W, self.wl.n_elec, 3))
            p = _dp(pos)
        self._check(self.L.qmc_init_walkers(self.h, self.W, p))

    def sweep(self, n: int = 1, count_accepted: bool = False) -> Optional[int]:
        if count_accepted:
            acc = C.c_uint64(0)
            self._check(self.L.qmc_sweep(self.h, int(n), C.byref(acc)))
            return int(acc.value)
        self._check(self.L.qmc_sweep(self.h, int(n), None))
        return None

    def measure(self, out=None) -> np.ndarray:
        """Local energies [W][4] (T, V_ee, V_eI, V_II).  With ``out`` a CUDA float64 tensor of
        shape [W, 4] the call is asynchronous and writes there."""
        if out is not None:
            self._check(self.L.qmc_measure_local_energy(self.h, C.c_void_p(out.data_ptr()), 1))
            return out
        e = np.zeros((self.W, 4))
        self._check(self.L.qmc_measure_local_energy(self.h, e.ctypes.data_as(C.c_void_p), 0))
        return e

    def run_steps(self, n: int, out):
        """n steps of (sweep + local energies), asynchronous; ``out`` a CUDA float64 tensor of
        shape [n, W, 4] receives every step's energies."""
        if tuple(out.shape) != (int(n), self.W, 4) or not out.is_contiguous():
            raise ValueError("out must be a contiguous [n, W, 4] tensor")
        self._check(self.L.qmc_run_steps(self.h, int(n), C.c_void_p(out.data_ptr())))
        return out

    def dmc_init(self, n_target: int, e_trial: float = float("nan"), feedback: float = 1.0):
        """Start a diffusion Monte Carlo population in the first ``n_target`` slots."""
        self._check(self.L.qmc_dmc_init(self.h, int(n_target), float(e_trial), float(feedback)))

    def dmc_steps(self, n: int, out):
        """n DMC steps, asynchronous; ``out`` a CUDA float64 tensor [n, 6] receives per step
        (E, sum of weights, population, E_T used, dropped copies, node-crossing rejections)."""
        if tuple(out.shape) != (int(n), 6) or not out.is_contiguous():
            raise ValueError("out must be a contiguous [n, 6] tensor")
        self._check(self.L.qmc_dmc_steps(self.h, int(n), C.c_void_p(out.data_ptr())))
        return out

    def dmc_state(self):
        """(weights[W], energies[W], E_T, population)."""
        w = np.zeros(self.W)
        e = np.zeros(self.W)
        et = C.c_double(0.0)
        pop = C.c_int32(0)
        self._check(self.L.qmc_dmc_get(self.h, w.ctypes.data_as(C.POINTER(C.c_double)),
                                       e.ctypes.data_as(C.POINTER(C.c_double)), C.byref(et), C.byref(pop)))
        return w, e, et.value, pop.value

    def set_sweep_index(self, index: int):
        """The index of the next sweep in the random streams (resume after init_pos)."""
        self._check(self.L.qmc_set_sweep_index(self.h, int(index)))

    def dmc_branching(self):
        """The last step's (weights before branching [W], energies [W], multiplicities [W],
        copy plan [W])."""
        w = np.zeros(self.W)
        e = np.zeros(self.W)
        m = np.zeros(self.W, dtype=np.int32)
        pl = np.zeros(self.W, dtype=np.int32)
        i32 = C.POINTER(C.c_int32)
        self._check(self.L.qmc_dmc_get_branching(self.h, _dp(w), _dp(e), m.ctypes.data_as(i32),
                                                 pl.ctypes.data_as(i32)))
        return w, e, m, pl

    def get_walkers(self):
        N = self.wl.n_elec
        pos = np.zeros((self.W, N, 3))
        ld = np.zeros((self.W, 2))
        sg = np.zeros((self.W, 2), dtype=np.int32)
        self._check(self.L.qmc_get_walkers(self.h, _dp(pos), _dp(ld), sg.ctypes.data_as(C.POINTER(C.c_int32))))
        return pos, ld, sg

    def accept_log(self) -> np.ndarray:
        bits = np.zeros((self.W, self.wl.n_elec), dtype=np.uint8)
        self._check(self.L.qmc_get_accept_log(self.h, bits.ctypes.data_as(C.POINTER(C.c_uint8))))
        return bits

    def counters(self):
        """(moves re-decided in FP64, sweeps run) since init_walkers."""
        a, b = C.c_uint64(0), C.c_uint64(0)
        self._check(self.L.qmc_get_counters(self.h, C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def precision_stats(self):
        """Mixed precision: (early FP64 rebuilds, walker sweeps run in FP64 fallback, walkers in
        fallback now, fallback mask [W]) since init_walkers."""
        a, b, c = C.c_uint64(0), C.c_uint64(0), C.c_int32(0)
        mask = np.zeros(self.W, dtype=np.int32)
        self._check(self.L.qmc_get_precision_stats(self.h, C.byref(a), C.byref(b), C.byref(c),
                                                   mask.ctypes.data_as(C.POINTER(C.c_int32))))
        return int(a.value), int(b.value), int(c.value), mask

    def recompute(self) -> np.ndarray:
        drift = np.zeros((self.W, 2))
        self._check(self.L.qmc_recompute(self.h, _dp(drift)))
        return drift

    def eval_spo_vgl(self, pos) -> np.ndarray:
        pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))
        out = np.zeros((pos.shape[0], 5, self.wl.n_orb))
        self._check(self.L.qmc_eval_spo_vgl(self.h, pos.shape[0], _dp(pos), _dp(out)))
        return out

    def eval_spo_vgl_noalloc(self, pos) -> np.ndarray:
        """As eval_spo_vgl, staged in the library's fixed device array (no device allocation)."""
        pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))
        out = np.zeros((pos.shape[0], 5, self.wl.n_orb))
        self._check(self.L.qmc_eval_spo_vgl_noalloc(self.h, pos.shape[0], _dp(pos), _dp(out)))
        return out

    def set_delay_rank(self, K: int):
        self._check(self.L.qmc_set_delay_rank(self.h, int(K)))

    def autotune_delay(self, ranks=(8, 16, 32, 64), trial_sweeps: int = 3):
        """Time the move chain with each delay rank (trial sweeps are ordinary sweeps); keep the best."""
        arr = (C.c_int32 * len(ranks))(*ranks)
        best = C.c_int32(0)
        ms = C.c_double(0.0)
        self._check(self.L.qmc_autotune_delay(self.h, arr, len(ranks), int(trial_sweeps), C.byref(best),
                                              C.byref(ms)))
        self.wl.delay_rank = int(best.value)
        return int(best.value), float(ms.value)

    def autotune_gather(self, trial_sweeps: int = 3):
        """Choose the gather's lanes per proposal by timing; returns (log2 lanes, gather ms)."""
        tl = C.c_int32(0)
        ms = C.c_double(0.0)
        self._check(self.L.qmc_autotune_gather(self.h, int(trial_sweeps), C.byref(tl), C.byref(ms)))
        return tl.value, ms.value

    def set_gather_lanes(self, lanes_log2: int):
        self._check(self.L.qmc_set_gather_lanes(self.h, int(lanes_log2)))

    def last_energies(self) -> np.ndarray:
        e = np.zeros((self.W, 4))
        self._check(self.L.qmc_get_last_energies(self.h, _dp(e)))
        return e

    def set_timing(self, on: bool = True):
        self._check(self.L.qmc_set_timing(self.h, int(bool(on))))

    def kernel_timing(self, kernel_class: int, reset: bool = False):
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        self._check(self.L.qmc_kernel_timing(self.h, kernel_class, C.byref(ms), C.byref(n), int(reset)))
        return ms.value, n.value


def estimate_device_bytes(wl, n_walkers: int) -> int:
    keep: list = []
    d = make_desc(wl, keep)
    g = wl.grid
    return int(load_library().qmc_estimate_device_bytes(C.byref(d), n_walkers, g[0], g[1], g[2]))


def max_delay_rank(wl) -> int:
    """Largest delay rank whose chain fits one workgroup's LDS (1: Sherman-Morrison only)."""
    keep: list = []
    k = int(load_library().qmc_max_delay_rank(C.byref(make_desc(wl, keep))))
    if k == 0:
        raise QMCError(QMC_ERR_ARG, "qmc_max_delay_rank rejected the descriptor")
    return k


class Batch:
    """Several initialised systems advanced by fused launches (see qmc_batch_* in include/qmc.h)."""

    def __init__(self, systems, stream=None, graph: bool = False):
        import torch
        self.L = load_library()
        self.systems = list(systems)
        if stream is None:
            stream = torch.cuda.Stream() if graph else torch.cuda.current_stream()
        self.stream = stream
        hs = (C.c_void_p * len(self.systems))(*[s.h.value for s in self.systems])
        b = C.c_void_p()
        st = self.L.qmc_batch_create(hs, len(self.systems), C.c_void_p(stream.cuda_stream), C.byref(b))
        if st != QMC_OK:
            raise QMCError(st, self.L.qmc_last_error(None).decode())
        self.b = b
        if graph:
            self._check(self.L.qmc_batch_set_graph(self.b, 1))

    def _check(self, st):
        if st != QMC_OK:
            raise QMCError(st, self.L.qmc_last_error(None).decode())

    def sweep(self, n: int = 1, measure: bool = False):
        self._check(self.L.qmc_batch_sweep(self.b, int(n), int(bool(measure))))

    def timing(self, reset: bool = False):
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        self._check(self.L.qmc_batch_timing(self.b, C.byref(ms), C.byref(n), int(reset)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "b", None):
            self.L.qmc_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
