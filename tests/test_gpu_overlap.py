"""Parity of the overlap histogram (int8 MFMA pair products) with the oracle:
bit-exact integer counts, including ragged batches and spin counts, the
all-configurations closed form, and exact first and second moments at the
benchmark size (16384 samples of 1000 spins)."""
import math

import numpy as np
import pytest
import torch

import paper_2606_22984_amd as fv
from oracle import overlap, physics
from tests.gpu_util import say, to_np
from workloads.instances import random_spins

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("B,N", [(1, 5), (2, 7), (64, 100), (65, 1000), (200, 33), (130, 64), (77, 16000)])
def test_overlap_histogram_matches_oracle(B, N):
    s = random_spins(B, N, B * 31 + N)
    say(f"overlap B={B} N={N}")
    got = to_np(fv.overlap_histogram(torch.as_tensor(s, device="cuda")))
    assert np.array_equal(got, overlap.overlap_counts(s))


def test_overlap_histogram_all_configurations():
    n = 12
    got = to_np(fv.overlap_histogram(torch.as_tensor(physics.all_configs(n), device="cuda")))
    assert got.tolist() == [2 ** (n - 1) * math.comb(n, k) for k in range(n)] + [0]


def test_overlap_histogram_moments_at_benchmark_size():
    B, N = 16384, 1000
    rng = np.random.default_rng(5)
    s = np.where(rng.random((B, N)) < 0.45, -1, 1).astype(np.int8)
    got = to_np(fv.overlap_histogram(torch.as_tensor(s, device="cuda"))).astype(np.int64)
    x = 2 * np.arange(N + 1, dtype=np.int64) - N        # s_a . s_b of each bin
    assert got.sum() == B * (B - 1) // 2
    col = s.astype(np.int64).sum(axis=0)
    m1 = (int((col * col).sum()) - B * N) // 2             # sum over a < b of s_a . s_b
    assert int((got * x).sum()) == m1
    f = s.astype(np.float64)
    G = f.T @ f                                            # exact: integer entries <= B
    m2 = (int(np.rint((G * G).sum())) - B * N * N) // 2    # sum over a < b of (s_a . s_b)^2
    assert int((got * x * x).sum()) == m2
