"""Learning-rate schedule of the learned-filter training driver (CPU): cosine
decay from the base rate at the first step towards zero at the last, or a
constant rate."""
import math
import os
import sys
from types import SimpleNamespace

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2104_13248_amd.train_learned import learning_rate  # noqa: E402


def test_cosine_schedule_decays_from_the_base_rate_to_zero():
    a = SimpleNamespace(lr=1e-3, schedule="cosine")
    total = 2000
    rates = [learning_rate(a, it, total) for it in range(total)]
    assert rates[0] == a.lr
    assert math.isclose(rates[total // 2], a.lr / 2, rel_tol=1e-12)
    assert 0.0 < rates[-1] < a.lr * 1e-5
    assert all(x >= y for x, y in zip(rates, rates[1:]))


def test_constant_schedule():
    a = SimpleNamespace(lr=2e-3, schedule="constant")
    assert {learning_rate(a, it, 100) for it in range(100)} == {2e-3}
