"""CPU-only checks of the C-ABI library: it loads, exports every symbol that
include/sg.h declares, and validates specifications (no GPU calls)."""
import os
import re

import numpy as np
import pytest

from paper_0704_3573_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "sg.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|int32_t|const char \*)\s*(sg_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTS) == names


def test_wheels_per_copy():
    for L, nw in ((2, 2), (4, 4), (8, 8), (16, 32), (24, 72), (32, 128), (48, 288), (64, 512)):
        assert B.wheels_per_copy(L) == nw
    assert B.wheels_per_copy(12) == 0 and B.wheels_per_copy(72) == 0
    # 4D glassy Potts: one wheel per (z, u, row group)
    for L, nw in ((2, 4), (4, 16), (8, 64), (16, 512)):
        assert B.wheels_per_copy(L, B.GPOTTS4) == nw
    assert B.wheels_per_copy(24, B.GPOTTS4) == 0


def test_glassy_potts_job_bytes():
    # one coupling word per site and sample (six permutation numbers) on top of
    # the +-J glass's one pattern byte per site
    g = B.job_bytes(B.Spec(B.GPOTTS, B.HEATBATH, 4, 16, 3, 2, 1, 0))
    p = B.job_bytes(B.Spec(B.POTTS, B.HEATBATH, 4, 16, 3, 2, 1, 0))
    assert g - p >= 3 * 3 * 16 ** 3 - 3 * 256


def test_ising_like_job_bytes():
    # 14 coupling words per (colour, block row, plane) and the occupancy copy,
    # on top of the EA glass's 6 words; one field sum per copy
    for L in (8, 16, 64):
        g = B.job_bytes(B.Spec(B.ISING_GEN, B.METROPOLIS, 4, L, 2, 2, 1, 0, 1.5))
        e = B.job_bytes(B.Spec(B.ISING, B.METROPOLIS, 4, L, 2, 2, 1, 0))
        assert g - e >= 2 * (8 * L ** 3 // 8 + L ** 3 // 8)
    # no parallel tempering, but several temperatures without it are fine
    assert B.job_bytes(B.Spec(B.ISING_GEN, B.HEATBATH, 4, 8, 1, 2, 4, 0, 0.0)) > 0
    assert B.job_bytes(B.Spec(B.ISING_GEN, B.HEATBATH, 4, 8, 1, 2, 1, 10, 0.0)) > 0


def test_4d_glassy_potts_job_bytes():
    # L = 16 in 4D: 65536 bytes of spins per copy, two coupling words per
    # site and sample, 512 wheels per copy
    b = B.job_bytes(B.Spec(B.GPOTTS4, B.HEATBATH, 4, 16, 2, 2, 1, 0))
    assert 4 * 16 ** 4 + 2 * 8 * 16 ** 4 + 4 * 512 * 64 * 4 < b < 3_000_000


def test_job_bytes_and_validation():
    n = B.job_bytes(B.Spec(B.ISING, B.METROPOLIS, 4, 64, 1, 2, 1, 0))
    # two copies of 64^3 bit-packed spins, shared couplings, 512 wheels x 64 slots each
    assert 2 * 64 ** 3 // 8 + 512 * 64 * 4 * 2 < n < 1_000_000
    for spec, code in (
        (B.Spec(B.ISING, B.METROPOLIS, 4, 12, 1, 1, 1, 0), B.SG_E_UNSUPPORTED),
        (B.Spec(B.POTTS, B.METROPOLIS, 4, 8, 1, 1, 1, 0), B.SG_E_UNSUPPORTED),
        (B.Spec(B.POTTS, B.HEATBATH, 3, 8, 1, 1, 1, 0), B.SG_E_UNSUPPORTED),
        (B.Spec(B.POTTS, B.HEATBATH, 4, 64, 1, 1, 1, 0), B.SG_E_UNSUPPORTED),
        (B.Spec(B.ISING, B.METROPOLIS, 4, 8, 0, 1, 1, 0), B.SG_E_INVALID),
        (B.Spec(B.ISING, 7, 4, 8, 1, 1, 1, 0), B.SG_E_INVALID),
        (B.Spec(B.ISING, B.METROPOLIS, 4, 8, 1, 1, 1, -1), B.SG_E_INVALID),
        (B.Spec(B.GPOTTS, B.METROPOLIS, 4, 8, 1, 1, 1, 0), B.SG_E_UNSUPPORTED),
        (B.Spec(B.GPOTTS, B.HEATBATH, 3, 8, 1, 1, 1, 0), B.SG_E_UNSUPPORTED),
        (B.Spec(B.GPOTTS, B.HEATBATH, 4, 56, 1, 1, 1, 0), B.SG_E_UNSUPPORTED),
        (B.Spec(B.ISING_GEN, B.METROPOLIS, 4, 8, 1, 1, 1, 0, -0.5), B.SG_E_INVALID),
        (B.Spec(B.ISING_GEN, B.HEATBATH, 4, 8, 1, 1, 1, 0, float("inf")), B.SG_E_INVALID),
        (B.Spec(B.ISING_GEN, B.HEATBATH, 4, 8, 1, 1, 1, 0, float("nan")), B.SG_E_INVALID),
        (B.Spec(B.ISING_GEN, B.METROPOLIS, 4, 8, 1, 2, 4, 10, 1.0), B.SG_E_UNSUPPORTED),
        (B.Spec(B.ISING_GEN, B.METROPOLIS, 4, 12, 1, 1, 1, 0, 1.0), B.SG_E_UNSUPPORTED),
        (B.Spec(B.GPOTTS4, B.METROPOLIS, 4, 8, 1, 1, 1, 0), B.SG_E_UNSUPPORTED),
        (B.Spec(B.GPOTTS4, B.HEATBATH, 4, 24, 1, 1, 1, 0), B.SG_E_UNSUPPORTED),
        (B.Spec(B.GPOTTS4, B.HEATBATH, 3, 8, 1, 1, 1, 0), B.SG_E_UNSUPPORTED),
        (B.Spec(5, B.HEATBATH, 4, 8, 1, 1, 1, 0), B.SG_E_INVALID),
    ):
        with pytest.raises(B.SgError) as e:
            B.job_bytes(spec)
        assert e.value.code == code
        assert B.lib().sg_last_error().decode()


MODEL_NAMES = {"ising": B.ISING, "potts": B.POTTS, "gpotts": B.GPOTTS, "gpotts4": B.GPOTTS4,
               "isinggen": B.ISING_GEN}


@pytest.mark.parametrize("name", sorted(MODEL_NAMES))
def test_library_generates_the_seeded_instances(name):
    """A job created from its seed alone gets exactly the inputs of the
    seeded-input module (couplings, spins, sweep and parallel-tempering
    wheels), numbered from the job's first sample."""
    from paper_0704_3573_amd import inputs
    model = MODEL_NAMES[name]
    Ls = (2, 4, 8) if name == "gpotts4" else (2, 4, 8, 16)
    for L in Ls:
        for S, R, K, seed, s0 in ((1, 1, 1, 1, 0), (2, 2, 3, 12345, 7)):
            algo = B.METROPOLIS if name in ("ising", "isinggen") else B.HEATBATH
            spec = B.Spec(model, algo, 4, L, S, R, K, 0, 0.0, seed, s0)
            got = B.generate(spec)
            want = inputs.make_instance(name, L, S, R, K, seed, s0)
            for key in ("J", "spins", "wheels", "ptwheels"):
                assert np.array_equal(got[key], want[key].reshape(got[key].shape)), (name, L, key)


def test_generate_rejects_bad_specs():
    with pytest.raises(B.SgError):
        B.generate(B.Spec(B.ISING, B.METROPOLIS, 4, 12, 1, 1, 1, 0))


def test_injected_device_error_is_reported_and_leaves_the_library_usable(monkeypatch):
    """The test hook makes a named entry point fail with SG_E_HIP at entry;
    the binding raises with that code and the thread's message, and the
    next call without the hook succeeds."""
    monkeypatch.setenv("SG_TEST_INJECT_HIP_ERROR", "sg_threshold_row")
    with pytest.raises(B.SgError) as e:
        B.threshold_row(B.ISING, B.METROPOLIS, 1.0)
    assert e.value.code == B.SG_E_HIP and "injected" in str(e.value)
    monkeypatch.setenv("SG_TEST_INJECT_HIP_ERROR", "sg_job_sweep")  # another entry point
    assert B.threshold_row(B.ISING, B.METROPOLIS, 1.0)[0] > 0
    monkeypatch.delenv("SG_TEST_INJECT_HIP_ERROR")
    assert B.threshold_row(B.ISING, B.METROPOLIS, 1.0)[0] > 0
