"""Host logic of the closure's rollout training: the order in which runs
visit the training seeds (no GPU)."""
import pytest

torch = pytest.importorskip("torch")

from paper_1402_5487_amd.closure_train import visit_order


def test_plain_order_is_a_permutation():
    o = visit_order(range(200), 8, seed=0)
    assert sorted(o) == list(range(200)) and o != list(range(200))
    assert o == visit_order(range(200), 8, seed=0)            # deterministic


@pytest.mark.parametrize("block,rounds", [(3, 5), (3, 3), (8, 3), (1, 2)])
def test_grouped_revisits(block, rounds):
    B = 8
    base = visit_order(range(200), B, seed=0)
    o = visit_order(range(200), B, seed=0, revisit=(block, rounds))
    assert len(o) == rounds * 200
    for s in range(200):
        pos = [i for i, x in enumerate(o) if x == s]
        assert len(pos) == rounds
        # consecutive visits of a seed lie block * B visits apart at most
        assert all(b - a <= block * B for a, b in zip(pos, pos[1:])), (s, pos)
    # every group of B consecutive visits is one group of the shuffled order
    groups = {tuple(base[i:i + B]) for i in range(0, 200, B)}
    assert all(tuple(o[i:i + B]) in groups for i in range(0, len(o), B))


def test_shipped_training_visits_each_seed_five_times():
    """2000 iterations of 8 runs x 32 steps, visits of 512 steps: exactly one
    pass over the revisit schedule, each of the 200 seeds five times."""
    iters, B, seg, visit = 2000, 8, 32, 512
    o = visit_order(range(200), B, seed=0, revisit=(3, 5))
    assert iters * B * seg // visit == len(o) == 1000
