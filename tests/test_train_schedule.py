"""The training driver's schedule against the oracle's (CPU)."""
import math

from oracle import optim as oo
from paper_2308_04079_amd.train import TrainConfig, Trainer


def test_trainer_schedule_equals_oracle_schedule():
    t = object.__new__(Trainer)
    t.cfg = TrainConfig()
    t.extent = 2.5
    t.max_deg = 3
    for it in list(range(0, 1200, 7)) + [2999, 3000, 3001, 6000, 14999, 15000, 15100, 29999, 30000]:
        assert t.resolution_divisor(it) == oo.resolution_divisor(it)
        assert t.sh_degree(it) == oo.sh_degree_at(it)
        assert t.densify_now(it) == oo.densify_now(it), it
        assert t.reset_now(it) == oo.reset_opacity_now(it)
        assert math.isclose(t.lr_means(it), 2.5 * oo.position_lr(it, 30000, 1.6e-4, 1.6e-6),
                            rel_tol=1e-12)
