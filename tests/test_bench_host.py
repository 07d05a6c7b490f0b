"""Host-side checks of bench.py: the algorithmic counts its roofline uses, by brute-force enumeration,
and its refusal of more than one GPU (no GPU needed)."""

import itertools
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _multi_indices(q):
    return [a for a in itertools.product(range(q + 1), repeat=3) if sum(a) <= q]


@pytest.mark.parametrize("q", [2, 4, 6, 8])
def test_interaction_flops_count_every_alpha_beta_pair(q):
    """One multiply-add per (alpha, beta) with |alpha| + |beta| <= q."""
    mi = _multi_indices(q)
    pairs = sum(1 for a in mi for b in mi if sum(a) + sum(b) <= q)
    assert bench.m2l_flops_per_pair(q) == 2 * pairs
    assert {4: 420, 6: 1848, 8: 6006}.get(q, 2 * pairs) == 2 * pairs


@pytest.mark.parametrize("q", [2, 4, 6, 8])
def test_reduced_flops_count_the_harmonic_triangle(q):
    """The kernels run the pairs with alpha_z <= 1 and beta_z <= 1 only."""
    mi = [a for a in _multi_indices(q) if a[2] <= 1]
    pairs = sum(1 for a in mi for b in mi if sum(a) + sum(b) <= q)
    assert bench.m2l_reduced_flops_per_pair(q) == 2 * pairs
    assert len(mi) == (q + 1) ** 2


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
