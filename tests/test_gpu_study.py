"""The batch-size scaling study (section 4's rules and their empirical test)
in a reduced configuration: it runs end to end on the library's own step
and its measurements have the properties that hold whatever the scene:
update norms grow with the effective learning rate (constant < square root
< linear at every batch size), every cosine is a valid one, and the
precision of the batch-mean gradient grows with the batch size."""
import math

import pytest
import torch

pytestmark = pytest.mark.gpu


def test_reduced_study_runs_and_orders():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_18533_amd import raster, scaling_study as S
    raster.init(0)
    c = S.StudyConfig(gaussians=30_000, views=16, res=96, pretrain_steps=40, images=32, batches=(8,),
                      variance_batches=(1, 4, 8), variance_trials=8)
    print("reduced scaling study", flush=True)
    res = S.run_study(c, log=lambda s: print(s, flush=True))
    lr = res["lr_rules"]
    for b in c.batches:
        r = [lr[k][b]["norm_ratio"] for k in ("constant", "sqrt", "linear")]
        assert r[0] < r[1] < r[2], r
        for rules in (res["lr_rules"], res["momentum_rules"]):
            for k in rules:
                assert -1.0 <= rules[k][b]["cosine"] <= 1.0 and math.isfinite(rules[k][b]["norm_ratio"])
    prec = res["gradient_precision"]
    assert prec[4] > prec[1] and prec[8] > prec[4]
