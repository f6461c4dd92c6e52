"""Per-step training metrics (train.StepLog): one JSON object per line with
the step count, loss and throughput since the previous record. Host logic
only; a stand-in trainer supplies the values a BatchedTrainer would."""
import json

import torch

from paper_2406_18533_amd import train


class _Trainer:
    def __init__(self):
        self.step_dev = torch.zeros(1, dtype=torch.int64)
        self.V, self.n, self.overflows = 16, 1000, 0
        self._loss = 0.5

    def loss(self):
        return self._loss


def test_step_log_appends_one_record_per_call(tmp_path):
    path = str(tmp_path / "steps.jsonl")
    log = train.StepLog(path, every=5)
    tr = _Trainer()
    tr.step_dev += 5
    r1 = log.write(tr, 5, 0.05)
    tr.step_dev += 5
    tr._loss, tr.overflows = 0.25, 1
    log.write(tr, 5, 0.1)
    lines = [json.loads(s) for s in open(path).read().splitlines()]
    assert lines[0] == r1
    assert [x["step"] for x in lines] == [5, 10] and [x["loss"] for x in lines] == [0.5, 0.25]
    assert abs(lines[0]["ms_per_step"] - 10.0) < 1e-9 and abs(lines[1]["views_per_s"] - 800.0) < 1e-6
    assert lines[1]["overflow_redos"] == 1 and lines[1]["gaussians"] == 1000
