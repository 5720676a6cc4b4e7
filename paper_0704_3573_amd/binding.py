"""ctypes binding of libsg.so (include/sg.h): argument marshalling only.

PyTorch supplies device memory (a uint8 tensor per job arena) and streams
(``torch.cuda.Stream.cuda_stream``); every step of the sweep runs in the
library's HIP kernels.  If the library has not been built this module raises
on first use: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SG_LIBRARY names another build of the same library (for example one whose
# host code is built with sanitizers, for the CPU checks)
LIB_PATH = os.environ.get("SG_LIBRARY") or os.path.join(HERE, "libsg.so")

ISING, POTTS, GPOTTS = 0, 1, 2  # GPOTTS: glassy Potts model (permutation couplings)
ISING_GEN = 3  # Ising-like model of Eq. 2 with dilution and field (RFIM, DAFF)
GPOTTS4 = 4  # glassy Potts model on the 4D hypercubic lattice
METROPOLIS, HEATBATH = 0, 1

SG_OK, SG_E_INVALID, SG_E_UNSUPPORTED, SG_E_NOMEM, SG_E_HIP, SG_E_STATE = 0, -1, -2, -3, -4, -5

# every symbol declared in include/sg.h
EXPORTS = (
    "sg_last_error", "sg_wheels_per_copy", "sg_model_wheels_per_copy", "sg_ctx_create", "sg_ctx_destroy", "sg_job_bytes",
    "sg_job_create", "sg_job_set_betas", "sg_job_sweep", "sg_job_measure", "sg_job_energies",
    "sg_job_field_sums", "sg_job_get_spins", "sg_job_get_wheels", "sg_job_get_perm", "sg_job_get_pt_accepts",
    "sg_job_sweeps_done", "sg_job_debug_rng", "sg_job_destroy", "sg_batch_create",
    "sg_batch_add", "sg_batch_remove", "sg_batch_set_block", "sg_batch_run", "sg_batch_block",
    "sg_batch_set_timing", "sg_batch_sweep_ms", "sg_batch_set_budget", "sg_batch_get_budget",
    "sg_batch_destroy", "sg_generate", "sg_threshold_row", "sg_pt_factors", "sg_job_sweep_beta",
    "sg_job_checkpoint_bytes", "sg_job_checkpoint", "sg_job_restore", "sg_batch_run_static",
    "sg_batch_set_period_cap", "sg_job_set_wheel_lanes", "sg_job_wheel_lanes",
)


class SgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsg error {code}: {msg}")
        self.code = code


class Spec(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "model", "algo", "q", "L", "n_samples", "n_replicas", "n_temps", "pt_every")] + [
        ("field", C.c_double), ("seed", C.c_uint64), ("sample0", C.c_uint64)]


_lib = None


def lib():
    """Load libsg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp, u64, i32 = C.c_void_p, C.c_uint64, C.c_int32
        L.sg_last_error.restype = C.c_char_p
        L.sg_wheels_per_copy.argtypes = [i32]
        L.sg_wheels_per_copy.restype = i32
        L.sg_model_wheels_per_copy.argtypes = [i32, i32]
        L.sg_model_wheels_per_copy.restype = i32
        L.sg_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
        L.sg_ctx_destroy.argtypes = [vp]
        L.sg_job_bytes.argtypes = [C.POINTER(Spec), C.POINTER(u64)]
        L.sg_job_create.argtypes = [vp, C.POINTER(Spec), vp, vp, vp, vp, vp, vp, u64, vp, u64, vp,
                                    C.POINTER(vp)]
        L.sg_job_set_betas.argtypes = [vp, vp, vp]
        L.sg_job_set_wheel_lanes.argtypes = [vp, C.c_int32, vp]
        L.sg_job_wheel_lanes.argtypes = [vp, C.POINTER(C.c_int32)]
        L.sg_job_sweep.argtypes = [vp, u64, vp]
        L.sg_job_measure.argtypes = [vp, vp, vp, vp]
        L.sg_job_energies.argtypes = [vp, vp, vp]
        L.sg_job_field_sums.argtypes = [vp, vp, vp]
        L.sg_job_get_spins.argtypes = [vp, vp, vp]
        L.sg_job_get_wheels.argtypes = [vp, vp, vp, vp]
        L.sg_job_get_perm.argtypes = [vp, vp, vp]
        L.sg_job_get_pt_accepts.argtypes = [vp, vp, vp]
        L.sg_job_sweeps_done.argtypes = [vp, C.POINTER(u64)]
        L.sg_job_debug_rng.argtypes = [vp, i32, i32, C.c_uint32, vp, vp]
        L.sg_job_destroy.argtypes = [vp]
        L.sg_batch_create.argtypes = [vp, vp, i32, C.POINTER(vp)]
        L.sg_generate.argtypes = [C.POINTER(Spec), vp, vp, vp, vp]
        L.sg_threshold_row.argtypes = [i32, i32, C.c_double, C.c_double, vp]
        L.sg_pt_factors.argtypes = [C.c_double, C.c_double, vp, C.POINTER(i32)]
        L.sg_job_sweep_beta.argtypes = [vp, C.c_double, u64, vp]
        L.sg_job_checkpoint_bytes.argtypes = [vp, C.POINTER(u64)]
        L.sg_job_checkpoint.argtypes = [vp, vp, u64, vp]
        L.sg_job_restore.argtypes = [vp, vp, u64, vp]
        L.sg_batch_add.argtypes = [vp, vp]
        L.sg_batch_remove.argtypes = [vp, vp]
        L.sg_batch_set_block.argtypes = [vp, i32]
        L.sg_batch_run.argtypes = [vp, u64, vp]
        L.sg_batch_run_static.argtypes = [vp, u64, vp]
        L.sg_batch_block.argtypes = [vp, C.POINTER(i32)]
        L.sg_batch_set_timing.argtypes = [vp, i32]
        L.sg_batch_sweep_ms.argtypes = [vp, C.POINTER(C.c_float)]
        L.sg_batch_set_budget.argtypes = [vp, vp, u64]
        L.sg_batch_get_budget.argtypes = [vp, vp, C.POINTER(u64)]
        L.sg_batch_set_period_cap.argtypes = [vp, vp, u64]
        L.sg_batch_destroy.argtypes = [vp]
        for n in EXPORTS:
            if n not in ("sg_last_error", "sg_wheels_per_copy", "sg_model_wheels_per_copy"):
                getattr(L, n).restype = C.c_int
        _lib = L
    return _lib


def _chk(rc):
    if rc != SG_OK:
        raise SgError(rc, lib().sg_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data


def _stream(stream):
    if stream is None:
        return None
    return C.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def wheels_per_copy(L: int, model: int = ISING) -> int:
    return int(lib().sg_model_wheels_per_copy(model, L))


def _rows(model) -> int:
    return {ISING_GEN: 5, GPOTTS4: 4}.get(model, 3)


def generate(spec: Spec):
    """The seeded instance of a specification, generated by the library
    (host only): dict with J, spins, wheels, ptwheels in canonical formats."""
    S, R, K = spec.n_samples, spec.n_replicas, spec.n_temps
    N = spec.L ** (4 if spec.model == GPOTTS4 else 3)
    NW = wheels_per_copy(spec.L, spec.model)
    ising = spec.model in (ISING, ISING_GEN)
    J = np.zeros((S, _rows(spec.model), N), np.uint8 if spec.model in (GPOTTS, GPOTTS4) else np.int8)
    spins = np.zeros((S * R * K, N), np.int8 if ising else np.uint8)
    wheels = np.zeros((S * R * K, NW, 61), np.uint32)
    ptwheels = np.zeros((S * R, 61), np.uint32)
    _chk(lib().sg_generate(C.byref(spec), _ptr(J), _ptr(spins), _ptr(wheels), _ptr(ptwheels)))
    return {"J": J, "spins": spins, "wheels": wheels, "ptwheels": ptwheels}


def threshold_row(model, algo, beta: float, field: float = 0.0) -> np.ndarray:
    """The 32-word integer threshold row the library uploads for one
    temperature (host only)."""
    row = np.zeros(32, np.uint32)
    _chk(lib().sg_threshold_row(model, algo, float(beta), float(field), _ptr(row)))
    return row


def pt_factors(beta_i: float, beta_next: float):
    """(F[24], sign) of the parallel-tempering pair (host only)."""
    F = np.zeros(24, np.uint64)
    sgn = C.c_int32()
    _chk(lib().sg_pt_factors(float(beta_i), float(beta_next), _ptr(F), C.byref(sgn)))
    return F, sgn.value


def job_bytes(spec: Spec) -> int:
    n = C.c_uint64()
    _chk(lib().sg_job_bytes(C.byref(spec), C.byref(n)))
    return n.value


class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _chk(lib().sg_ctx_create(device, C.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().sg_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Job:
    """One job: S samples x R replicas x K temperature slots of one (model, L).

    Device state lives in a torch uint8 tensor (the arena) owned by this
    object.  Arrays follow the canonical formats of include/sg.h.
    """

    def __init__(self, ctx: Context, model, algo, L, betas, J=None, spins=None, wheels=None,
                 ptwheels=None, *, n_samples=1, n_replicas=1, pt_every=0, slot_of_temp=None,
                 sweeps_done=0, stream=None, arena=None, field=0.0, seed=0, sample0=0):
        """J, spins, wheels, ptwheels: canonical arrays, or None to have the
        library generate them from (seed, sample0)."""
        import torch
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        K = betas.shape[0]
        self.spec = Spec(model, algo, 4, L, n_samples, n_replicas, K, pt_every, float(field),
                         int(seed), int(sample0))
        self.model, self.algo, self.L = model, algo, L
        self.S, self.R, self.K = n_samples, n_replicas, K
        self.C = n_samples * n_replicas * K
        self.N = L ** (4 if model == GPOTTS4 else 3)
        self.NW = wheels_per_copy(L, model)
        self.bytes = job_bytes(self.spec)
        if arena is None:
            arena = torch.empty(self.bytes, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        self.arena = arena
        # +-1 couplings as int8; glassy-Potts permutation bytes as uint8 (same
        # width); Ising-like models: rows J_x, J_y, J_z, x, f
        self.ising_spins = model in (ISING, ISING_GEN)
        if J is not None:
            J = np.ascontiguousarray(J, dtype=np.uint8 if model in (GPOTTS, GPOTTS4) else np.int8)
            assert J.size == self.S * _rows(model) * self.N
        if spins is not None:
            spins = np.ascontiguousarray(spins, dtype=np.int8 if self.ising_spins else np.uint8)
            assert spins.size == self.C * self.N
        if wheels is not None:
            wheels = np.ascontiguousarray(wheels, dtype=np.uint32)
            assert wheels.size == self.C * self.NW * 61
        pw = None if ptwheels is None else np.ascontiguousarray(ptwheels, dtype=np.uint32)
        if pw is not None:
            assert pw.size == self.S * self.R * 61
        sot = None if slot_of_temp is None else np.ascontiguousarray(slot_of_temp, dtype=np.int32)
        h = C.c_void_p()
        _chk(lib().sg_job_create(ctx.h, C.byref(self.spec), _ptr(betas), _ptr(J), _ptr(spins),
                                 _ptr(wheels), _ptr(pw), _ptr(sot), sweeps_done,
                                 C.c_void_p(arena.data_ptr()), arena.numel(), _stream(stream),
                                 C.byref(h)))
        self.h = h
        self.ctx = ctx

    def close(self):
        if getattr(self, "h", None):
            lib().sg_job_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_betas(self, betas, stream=None):
        b = np.ascontiguousarray(betas, dtype=np.float64)
        _chk(lib().sg_job_set_betas(self.h, _ptr(b), _stream(stream)))

    def sweep(self, n: int, stream=None):
        _chk(lib().sg_job_sweep(self.h, n, _stream(stream)))

    def set_wheel_lanes(self, lanes: int, stream=None):
        _chk(lib().sg_job_set_wheel_lanes(self.h, int(lanes), _stream(stream)))

    def wheel_lanes(self) -> int:
        n = C.c_int32()
        _chk(lib().sg_job_wheel_lanes(self.h, C.byref(n)))
        return n.value

    def sweep_beta(self, beta: float, n: int, stream=None):
        _chk(lib().sg_job_sweep_beta(self.h, float(beta), n, _stream(stream)))

    def checkpoint(self, stream=None) -> bytes:
        n = C.c_uint64()
        _chk(lib().sg_job_checkpoint_bytes(self.h, C.byref(n)))
        buf = np.zeros(n.value, np.uint8)
        _chk(lib().sg_job_checkpoint(self.h, _ptr(buf), n.value, _stream(stream)))
        return buf.tobytes()

    def restore(self, blob: bytes, stream=None):
        buf = np.frombuffer(blob, np.uint8).copy()
        _chk(lib().sg_job_restore(self.h, _ptr(buf), buf.size, _stream(stream)))

    def measure(self, stream=None, overlap=True):
        E = np.zeros(self.C, dtype=np.int64)
        Q = np.zeros(self.S * self.K, dtype=np.int64) if (overlap and self.R >= 2) else None
        _chk(lib().sg_job_measure(self.h, _ptr(E), _ptr(Q), _stream(stream)))
        return E, Q

    def energies(self, stream=None):
        E = np.zeros(self.C, dtype=np.int64)
        _chk(lib().sg_job_energies(self.h, _ptr(E), _stream(stream)))
        return E

    def field_sums(self, stream=None):
        M = np.zeros(self.C, dtype=np.int64)
        _chk(lib().sg_job_field_sums(self.h, _ptr(M), _stream(stream)))
        return M

    def spins(self, stream=None):
        out = np.zeros((self.C, self.N), dtype=np.int8 if self.ising_spins else np.uint8)
        _chk(lib().sg_job_get_spins(self.h, _ptr(out), _stream(stream)))
        return out

    def wheels(self, stream=None):
        w = np.zeros((self.C, self.NW, 61), dtype=np.uint32)
        pw = np.zeros((self.S * self.R, 61), dtype=np.uint32)
        _chk(lib().sg_job_get_wheels(self.h, _ptr(w), _ptr(pw), _stream(stream)))
        return w, pw

    def perm(self, stream=None):
        out = np.zeros((self.S * self.R, self.K), dtype=np.int32)
        _chk(lib().sg_job_get_perm(self.h, _ptr(out), _stream(stream)))
        return out

    def pt_accepts(self, stream=None):
        out = np.zeros((self.S * self.R, max(self.K - 1, 1)), dtype=np.uint64)
        _chk(lib().sg_job_get_pt_accepts(self.h, _ptr(out), _stream(stream)))
        return out

    def sweeps_done(self) -> int:
        n = C.c_uint64()
        _chk(lib().sg_job_sweeps_done(self.h, C.byref(n)))
        return n.value

    def debug_rng(self, copy: int, wheel: int, n: int, stream=None):
        out = np.zeros(n, dtype=np.uint32)
        _chk(lib().sg_job_debug_rng(self.h, copy, wheel, n, _ptr(out), _stream(stream)))
        return out


class Batch:
    """Jobs advanced together by one fused launch per period (hipGraph replay)."""

    def __init__(self, ctx: Context, jobs=(), block: int = 0):
        jobs = list(jobs)
        hs = (C.c_void_p * max(1, len(jobs)))(*[j.h for j in jobs])
        h = C.c_void_p()
        _chk(lib().sg_batch_create(ctx.h, hs if jobs else None, len(jobs), C.byref(h)))
        self.h = h
        self.jobs = jobs
        if block:
            self.set_block(block)

    def add(self, job: Job):
        _chk(lib().sg_batch_add(self.h, job.h))
        self.jobs.append(job)

    def remove(self, job: Job):
        _chk(lib().sg_batch_remove(self.h, job.h))
        self.jobs.remove(job)

    def set_block(self, threads: int):
        _chk(lib().sg_batch_set_block(self.h, threads))

    def block(self) -> int:
        n = C.c_int32()
        _chk(lib().sg_batch_block(self.h, C.byref(n)))
        return n.value

    def run(self, n: int, stream=None):
        _chk(lib().sg_batch_run(self.h, n, _stream(stream)))

    def run_static(self, n: int, stream=None):
        """As run(), with the launch tables in the library's static device
        scratch: no device allocation (see sg_batch_run_static)."""
        _chk(lib().sg_batch_run_static(self.h, n, _stream(stream)))

    def set_budget(self, job: Job, sweeps: int):
        _chk(lib().sg_batch_set_budget(self.h, job.h, sweeps))

    def set_period_cap(self, job: Job, sweeps: int):
        _chk(lib().sg_batch_set_period_cap(self.h, job.h, sweeps))

    def budget(self, job: Job) -> int:
        n = C.c_uint64()
        _chk(lib().sg_batch_get_budget(self.h, job.h, C.byref(n)))
        return n.value

    def set_timing(self, on: bool):
        _chk(lib().sg_batch_set_timing(self.h, int(on)))

    def sweep_ms(self) -> float:
        ms = C.c_float()
        _chk(lib().sg_batch_sweep_ms(self.h, C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "h", None):
            lib().sg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
