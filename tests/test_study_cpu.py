"""Host logic of the batch-size scaling study: the hyperparameters handed
to the fused Adam (which applies lr sqrt(b) and beta^b, section 4 eqs.
"lambda" and "beta") give the named effective rules."""
import math

import pytest

from paper_2406_18533_amd import scaling_study as S


@pytest.mark.parametrize("b", [1, 4, 16, 32])
def test_rules_reach_the_named_effective_hyperparameters(b):
    base = [1e-3, 2e-3, 3e-3, 4e-3, 5e-3, 6e-3]
    want_lr = {"constant": 1.0, "sqrt": math.sqrt(b), "linear": float(b)}
    for rule, f in want_lr.items():
        lr6, b1, b2 = S.rule_hparams(base, 0.9, 0.999, b, rule, "exp")
        for x, y in zip(lr6, base):
            assert abs(x * math.sqrt(b) - y * f) <= 1e-15 * y * f
        assert (b1, b2) == (0.9, 0.999)                     # the kernel raises them to the b-th power
    _, b1, b2 = S.rule_hparams(base, 0.9, 0.999, b, "sqrt", "unchanged")
    assert abs(b1 ** b - 0.9) < 1e-14 and abs(b2 ** b - 0.999) < 1e-14


def test_compare_is_cosine_and_norm_ratio():
    import torch
    a = torch.tensor([3.0, 4.0, 0.0])
    r = torch.tensor([0.0, 4.0, 3.0])
    out = S.compare(a, r)
    assert abs(out["cosine"] - 16.0 / 25.0) < 1e-7 and abs(out["norm_ratio"] - 1.0) < 1e-7


def test_precision_correction_for_drawing_distinct_views():
    """Mean of b of V fixed gradients drawn without replacement: over all
    b-subsets, the variance of the mean is (sigma^2 / b) (V - b) / (V - 1)
    with sigma^2 the population variance (finite population correction), so
    the corrected precision is exactly b / mean(sigma^2): b times that of one
    view. A wrong correction factor fails the ratio."""
    import numpy as np
    import torch
    rng = np.random.default_rng(5)
    V = 7
    G = torch.from_numpy(rng.normal(size=(V, 50)) * rng.uniform(0.5, 2.0, size=50))
    out = S.precision_by_batch(G, range(1, V + 1), exhaustive=True)
    assert sorted(out) == list(range(1, V))           # b = V has no spread to measure
    sigma2 = G.numpy().var(axis=0, ddof=0).mean()
    assert out[1] == pytest.approx(1.0 / sigma2, rel=1e-12)
    for b in range(2, V):
        assert out[b] / out[1] == pytest.approx(b, rel=1e-12)
    # random draws estimate the same thing
    gen = torch.Generator().manual_seed(0)
    est = S.precision_by_batch(G, (3,), trials=4000, gen=gen)
    assert est[3] == pytest.approx(out[3], rel=0.1)
