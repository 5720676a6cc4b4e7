"""CPU oracle for the checkerboard spin-glass sweep -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library never does; the two
share no code (only the seeded input generators are common).

The arithmetic lives in ``sg_oracle.c`` (plain C, built with gcc); this
module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sg_oracle.c")
# SG_ORACLE_LIBRARY names another build of the oracle (a sanitizer build)
LIB = os.environ.get("SG_ORACLE_LIBRARY") or os.path.join(HERE, "liboracle.so")

ISING, POTTS, GPOTTS = 0, 1, 2  # GPOTTS: glassy (permutation) Potts, Eq. (3)
GPOTTS4 = 4  # glassy Potts model on the 4D hypercubic lattice
ISING_GEN = 3  # Ising-like model of Eq. (2) with dilution and field (RFIM, DAFF)
METROPOLIS, HEATBATH = 0, 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Spec(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "model", "algo", "L", "n_samples", "n_replicas", "n_temps",
        "pt_every", "measure_every", "check_energy", "n_threads")] + [("field", C.c_double)]


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        _lib = C.CDLL(LIB)
        u32p, u64p, i64p = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), C.POINTER(C.c_int64)
        _lib.or_pr_stream.argtypes = [u32p, C.c_uint64, u32p]
        for n, k in (("or_tables_metropolis", 3), ("or_tables_heatbath", 7), ("or_tables_potts", 13)):
            getattr(_lib, n).argtypes = [C.c_double, u64p]
        _lib.or_tables_pt.argtypes = [C.c_double, C.c_double, u64p]
        _lib.or_pt_threshold.argtypes = [u64p, C.c_uint64]
        _lib.or_pt_threshold.restype = C.c_uint64
        _lib.or_ising_update_site.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                              C.c_int64, C.c_uint32, u64p]
        _lib.or_ising_update_site.restype = C.c_int32
        _lib.or_potts_update_site.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                              C.c_uint32, u64p]
        _lib.or_potts_update_site.restype = C.c_int32
        _lib.or_gpotts_update_site.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                               C.c_uint32, u64p]
        _lib.or_gpotts_update_site.restype = C.c_int32
        _lib.or_gpotts_fields.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                          C.POINTER(C.c_int32)]
        _lib.or_gpotts4_update_site.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                                C.c_uint32, u64p]
        _lib.or_gpotts4_update_site.restype = C.c_int32
        _lib.or_gpotts4_fields.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                           C.POINTER(C.c_int32)]
        _lib.or_wheels_per_copy_4d.argtypes = [C.c_int32]
        _lib.or_wheels_per_copy_4d.restype = C.c_int32
        for n in ("or_ising_energy", "or_potts_energy", "or_gpotts_energy", "or_gpotts4_energy"):
            getattr(_lib, n).argtypes = [C.c_int32, C.c_void_p, C.c_void_p]
            getattr(_lib, n).restype = C.c_int64
        for n in ("or_ising_overlap", "or_potts_overlap"):
            getattr(_lib, n).argtypes = [C.c_int32, C.c_void_p, C.c_void_p]
            getattr(_lib, n).restype = C.c_int64
        _lib.or_isinggen_update_site.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                                 C.c_double, C.c_double, C.c_int64, C.c_uint32,
                                                 i64p]
        _lib.or_isinggen_update_site.restype = C.c_int32
        for n in ("or_isinggen_bond_energy", "or_isinggen_field_sum"):
            getattr(_lib, n).argtypes = [C.c_int32, C.c_void_p, C.c_void_p]
            getattr(_lib, n).restype = C.c_int64
        _lib.or_isinggen_overlap.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.or_isinggen_overlap.restype = C.c_int64
        _lib.or_wheels_per_copy.argtypes = [C.c_int32]
        _lib.or_wheels_per_copy.restype = C.c_int32
        _lib.or_run.argtypes = [C.POINTER(Spec), C.POINTER(C.c_double), C.c_void_p, C.c_void_p,
                                u32p, u32p, C.POINTER(C.c_int32), C.c_uint64, C.c_uint64,
                                i64p, i64p, i64p, u64p, i64p]
        _lib.or_run.restype = C.c_int32
    return _lib


# ---------------------------------------------------------------- RNG ----

def pr_stream(words, n: int) -> np.ndarray:
    """n Parisi-Rapuano outputs of a wheel given by its 61 words (oldest first)."""
    w = np.ascontiguousarray(words, dtype=np.uint32)
    assert w.shape == (61,)
    out = np.empty(n, dtype=np.uint32)
    lib().or_pr_stream(_p(w, C.c_uint32), n, _p(out, C.c_uint32))
    return out


# ------------------------------------------------------------- tables ----

def tables_metropolis(beta: float) -> np.ndarray:
    T = np.zeros(3, dtype=np.uint64)
    lib().or_tables_metropolis(beta, _p(T, C.c_uint64))
    return T


def tables_heatbath(beta: float) -> np.ndarray:
    T = np.zeros(7, dtype=np.uint64)
    lib().or_tables_heatbath(beta, _p(T, C.c_uint64))
    return T


def tables_potts(beta: float) -> np.ndarray:
    W = np.zeros(13, dtype=np.uint64)
    lib().or_tables_potts(beta, _p(W, C.c_uint64))
    return W


def tables_pt(beta_a: float, beta_b: float) -> np.ndarray:
    F = np.zeros(24, dtype=np.uint64)
    lib().or_tables_pt(beta_a, beta_b, _p(F, C.c_uint64))
    return F


def pt_threshold(F, absD: int) -> int:
    F = np.ascontiguousarray(F, dtype=np.uint64)
    return int(lib().or_pt_threshold(_p(F, C.c_uint64), absD))


# -------------------------------------------------------- single site ----

def ising_update_site(L, algo, s, J, i, r, T) -> int:
    """Update site i of int8 spins s in place with number r; returns dE."""
    T = np.ascontiguousarray(T, dtype=np.uint64)
    assert s.dtype == np.int8 and J.dtype == np.int8 and s.flags.c_contiguous
    return int(lib().or_ising_update_site(L, algo, s.ctypes.data, J.ctypes.data, i, r,
                                          _p(T, C.c_uint64)))


def potts_update_site(L, s, J, i, r, W) -> int:
    W = np.ascontiguousarray(W, dtype=np.uint64)
    assert s.dtype == np.uint8 and J.dtype == np.int8 and s.flags.c_contiguous
    return int(lib().or_potts_update_site(L, s.ctypes.data, J.ctypes.data, i, r,
                                          _p(W, C.c_uint64)))


def gpotts_update_site(L, s, P, i, r, W) -> int:
    """Glassy Potts: update site i of uint8 spins s with permutation bytes P [3][N]."""
    W = np.ascontiguousarray(W, dtype=np.uint64)
    assert s.dtype == np.uint8 and P.dtype == np.uint8 and s.flags.c_contiguous
    return int(lib().or_gpotts_update_site(L, s.ctypes.data, P.ctypes.data, i, r,
                                           _p(W, C.c_uint64)))


def gpotts_fields(L, s, P, i) -> np.ndarray:
    """Local fields h_a (a = 0..3) of site i of the glassy Potts model."""
    s = np.ascontiguousarray(s, dtype=np.uint8)
    P = np.ascontiguousarray(P, dtype=np.uint8)
    h = np.zeros(4, dtype=np.int32)
    lib().or_gpotts_fields(L, s.ctypes.data, P.ctypes.data, i, _p(h, C.c_int32))
    return h


def gpotts4_update_site(L, s, P, i, r, W) -> int:
    """4D glassy Potts: update site i of uint8 spins s (L^4) with P [4][N]."""
    W = np.ascontiguousarray(W, dtype=np.uint64)
    assert s.dtype == np.uint8 and P.dtype == np.uint8 and s.flags.c_contiguous
    return int(lib().or_gpotts4_update_site(L, s.ctypes.data, P.ctypes.data, i, r,
                                            _p(W, C.c_uint64)))


def gpotts4_fields(L, s, P, i) -> np.ndarray:
    """Local fields h_a (a = 0..3) of site i of the 4D glassy Potts model."""
    s = np.ascontiguousarray(s, dtype=np.uint8)
    P = np.ascontiguousarray(P, dtype=np.uint8)
    h = np.zeros(4, dtype=np.int32)
    lib().or_gpotts4_fields(L, s.ctypes.data, P.ctypes.data, i, _p(h, C.c_int32))
    return h


def isinggen_update_site(L, algo, s, D, field, beta, i, r):
    """General Ising-like model: update site i of int8 spins s (D = [5][N]);
    returns (change of the bond energy, change of the field sum)."""
    assert s.dtype == np.int8 and D.dtype == np.int8 and s.flags.c_contiguous
    dM = np.zeros(1, dtype=np.int64)
    dE = lib().or_isinggen_update_site(L, algo, s.ctypes.data, D.ctypes.data, field, beta, i, r,
                                       _p(dM, C.c_int64))
    return int(dE), int(dM[0])


def isinggen_terms(L, s, D):
    """(E_b, M): bond energy and field sum; H = E_b - field * M."""
    s = np.ascontiguousarray(s, dtype=np.int8)
    D = np.ascontiguousarray(D, dtype=np.int8)
    return (int(lib().or_isinggen_bond_energy(L, s.ctypes.data, D.ctypes.data)),
            int(lib().or_isinggen_field_sum(L, s.ctypes.data, D.ctypes.data)))


def _couplings(model, J):
    return np.ascontiguousarray(J, dtype=np.uint8 if model in (GPOTTS, GPOTTS4) else np.int8)


def energy(model, L, s, J) -> int:
    s = np.ascontiguousarray(s)
    J = _couplings(model, J)
    f = {ISING: lib().or_ising_energy, POTTS: lib().or_potts_energy,
         GPOTTS: lib().or_gpotts_energy, GPOTTS4: lib().or_gpotts4_energy}[model]
    return int(f(L, s.ctypes.data, J.ctypes.data))


def overlap(model, L, a, b) -> int:
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    f = lib().or_ising_overlap if model == ISING else lib().or_potts_overlap
    return int(f(L, a.ctypes.data, b.ctypes.data))


def wheels_per_copy(L: int, model: int = ISING) -> int:
    if model == GPOTTS4:
        return int(lib().or_wheels_per_copy_4d(L))
    return int(lib().or_wheels_per_copy(L))


# ---------------------------------------------------------------- run ----

class OracleError(RuntimeError):
    pass


def run(model, algo, L, betas, J, spins, wheels, ptwheels=None, slot_of_temp=None, *,
        n_samples=1, n_replicas=1, n_sweeps=0, sweeps_done=0, pt_every=0,
        measure_every=0, check_energy=False, n_threads=1, field=0.0):
    """Run the oracle; arrays are copied, the new state is returned.

    Returns a dict with spins, wheels, ptwheels, slot_of_temp, E (final, per
    slot), E_log [n_meas][C], Q_log [n_meas][S][K], pt_accepts [S*R][K-1] and
    M (final field sum per slot; ISING_GEN, whose E is the bond energy).
    """
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    K = betas.shape[0]
    S, R = n_samples, n_replicas
    Cn = S * R * K
    dim = 4 if model == GPOTTS4 else 3
    N = L ** dim
    NW = wheels_per_copy(L, model)
    J = _couplings(model, J).reshape(S, {ISING_GEN: 5, GPOTTS4: 4}.get(model, 3), N)
    sp = np.array(spins, dtype=np.int8 if model in (ISING, ISING_GEN) else np.uint8,
                  copy=True).reshape(Cn, N)
    wh = np.array(wheels, dtype=np.uint32, copy=True).reshape(Cn, NW, 61)
    if ptwheels is None:
        ptwheels = np.zeros((S * R, 61), dtype=np.uint32)
    pw = np.array(ptwheels, dtype=np.uint32, copy=True).reshape(S * R, 61)
    if slot_of_temp is None:
        slot_of_temp = np.tile(np.arange(K, dtype=np.int32), (S * R, 1))
    sot = np.array(slot_of_temp, dtype=np.int32, copy=True).reshape(S * R, K)
    n_meas = n_sweeps // measure_every if measure_every else 0
    E = np.zeros(Cn, dtype=np.int64)
    M = np.zeros(Cn, dtype=np.int64)
    E_log = np.zeros((max(n_meas, 1), Cn), dtype=np.int64)
    Q_log = np.zeros((max(n_meas, 1), S, K), dtype=np.int64)
    acc = np.zeros((S * R, max(K - 1, 1)), dtype=np.uint64)
    spec = Spec(model, algo, L, S, R, K, pt_every, measure_every, int(check_energy), n_threads,
                float(field))
    rc = lib().or_run(C.byref(spec), _p(betas, C.c_double), J.ctypes.data, sp.ctypes.data,
                      _p(wh, C.c_uint32), _p(pw, C.c_uint32), _p(sot, C.c_int32),
                      sweeps_done, n_sweeps, _p(E, C.c_int64), _p(E_log, C.c_int64),
                      _p(Q_log, C.c_int64), _p(acc, C.c_uint64), _p(M, C.c_int64))
    if rc != 0:
        raise OracleError(f"or_run failed with code {rc}")
    return {"spins": sp, "wheels": wh, "ptwheels": pw, "slot_of_temp": sot, "E": E,
            "E_log": E_log[:n_meas], "Q_log": Q_log[:n_meas], "pt_accepts": acc, "M": M}
