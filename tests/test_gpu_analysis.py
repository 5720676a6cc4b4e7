"""GPU parity of the equilibration analysis (sec. 4.1): overlaps measured by
libsg during a run, analysed by the library's analysis module, equal the
oracle's analysis of the oracle's own measurements of the same seeded run
(q^2 history and log2 bins to rounding, P(q) counts exactly)."""
import numpy as np
import pytest

import oracle
from oracle import analysis as OA
from paper_0704_3573_amd import analysis as PA
from tests._gpu import instance, make_job, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0704_3573_amd import binding as B
    return B.Context(0)


CASES = [
    # model, algo, L, S, K, pt_every, field, measure_every, measurements
    ("ising", oracle.METROPOLIS, 8, 4, 4, 5, 0.0, 5, 32),
    ("potts", oracle.HEATBATH, 8, 3, 1, 0, 0.0, 2, 24),
    ("daff", oracle.METROPOLIS, 16, 3, 2, 0, 1.1, 3, 20),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_analysis_of_gpu_measurements_equals_oracle(ctx, case):
    kind, algo, L, S, K, pe, h, every, n = CASES[case]
    betas = list(1 / np.linspace(0.8, 1.6, K)) if K > 1 else [1 / 1.1]
    inst = instance(kind, L, S=S, R=2, K=K, seed=600 + case)
    job = make_job(ctx, kind, algo, L, betas, inst, S=S, R=2, pt_every=pe, field=h)
    Qs = []
    for _ in range(n):
        job.sweep(every)
        Qs.append(job.measure()[1])
    model = job.model
    Q = PA.stack_measurements(Qs, S, K)
    N = PA.sites_per_sample(model, L, inst["J"])
    ref = run_oracle(kind, algo, L, betas, inst, S=S, R=2, n=n * every, pt_every=pe,
                     measure_every=every, field=h)
    Nl = [int(x) for x in N]
    Ql = ref["Q_log"].tolist()
    np.testing.assert_allclose(PA.q2_history(model, Q, N), OA.q2_history(model, Ql, Nl), rtol=1e-12)
    m, _ = PA.log2_binning(model, Q, N)
    np.testing.assert_allclose(m, [[x[0] for x in g] for g in OA.log2_bins(model, Ql, Nl)],
                               rtol=1e-12)
    c = PA.pq_counts(model, Q, N, start=n // 2)
    assert np.array_equal(c, np.array(OA.pq_counts(model, Ql, Nl, start=n // 2)))
