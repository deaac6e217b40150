"""CPU checks of the benchmark's byte accounting (the roofline numerator)
and of its one-GPU contract."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _info(**kw):
    base = dict(n_u=30, n_l=6, nnz_G=12, nnz_K=300, k_bs=3, k_blocks=40, k_index_bytes=2,
                k_lower_blocks=18, k_nnz_stored=170, k_slots=44 * 64)
    base.update(kw)
    return base


def test_smooth_u_bytes_full_layout():
    # vectors: 4 n_u-vectors + z_l, G CSR (value + column), row pointers
    vec = 30 * 4 * 4 + 6 * 4 + 12 * 8 + 31 * 4
    alg, stored = bench.smooth_u_bytes(_info(k_layout=1), 290, 4)
    assert alg == 290 * 4 + 40 * 2 + vec
    assert stored == 40 * (9 * 4 + 2) + vec


def test_smooth_u_bytes_symmetric_storage():
    # 22 stored blocks (2-byte delta each) holding 170 nonzeros, 18 mirrors
    # (2-byte delta + 2-byte position each)
    vec = 30 * 4 * 4 + 6 * 4 + 12 * 8 + 31 * 4
    alg, stored = bench.smooth_u_bytes(_info(k_layout=3), 290, 4)
    assert alg == 170 * 4 + 22 * 2 + 18 * 4 + vec
    assert stored == 22 * 9 * 4 + 22 * 2 + 18 * 4 + vec
    full = bench.smooth_u_bytes(_info(k_layout=1), 290, 4)[0]
    assert alg < full


def test_smooth_u_bytes_csr():
    b = 300 * (8 + 4) + 31 * 4 + (30 * 8 * 4 + 6 * 8 + 12 * 12 + 31 * 4)
    assert bench.smooth_u_bytes(_info(k_layout=0), 290, 8) == (b, b)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
