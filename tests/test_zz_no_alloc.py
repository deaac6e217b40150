"""The allocation-free V-cycle entry point (amg_vcycle_apply_noalloc) against
amg_vcycle_apply, through the C-ABI.

Both run the same kernels in the same order on the same hierarchy, and the
kernels are deterministic (no atomics), so the outputs must agree bit for
bit.  The calls alternate between a large and a small handle, so each call
finds the scratch array holding the previous call's (larger) contents.  The
small case is also compared with the oracle's V-cycle (FP64 1e-12, mixed
2e-5 relative).  A problem whose work vectors exceed the scratch array is
rejected before anything runs, and its handle keeps working.
"""
import numpy as np
import pytest
import torch

from contactgen import make_contact_problem, make_workload
from oracle.hierarchy import AMGOptions as OracleOptions
from oracle.hierarchy import build_hierarchy
from oracle.vcycle import vcycle as oracle_vcycle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_09056_amd.camg import load_library

    load_library()


def _solver(prob, precision, **kw):
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver

    return AMGSolver.from_problem(prob, AMGOptions(precision=precision, **kw))


def _noalloc(s, r, transpose):
    z = torch.full_like(r, float("nan"))
    s.vcycle_noalloc(r, z, transpose=transpose)
    torch.cuda.synchronize()
    return z


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_vcycle_matches_vcycle_apply(prec):
    big = make_workload("contact3d_40")
    small = make_workload("contact3d_6")
    sb = _solver(big, prec, max_levels=4)
    ss = _solver(small, prec, max_levels=2)
    rng = np.random.default_rng(11)
    rb = torch.from_numpy(rng.standard_normal(big.n)).cuda()
    rs = torch.from_numpy(rng.standard_normal(small.n)).cuda()
    lv = build_hierarchy(small, OracleOptions(max_levels=2))
    tol = 1e-12 if prec == 0 else 2e-5
    for tr in (False, True):
        print(f"[noalloc] prec={prec} transpose={tr} 40^3 then 6^3 then 40^3", flush=True)
        zb = _noalloc(sb, rb, tr)
        zs = _noalloc(ss, rs, tr)
        zb2 = _noalloc(sb, rb, tr)
        ref_b = sb.vcycle(rb, transpose=tr)
        ref_s = ss.vcycle(rs, transpose=tr)
        torch.cuda.synchronize()
        assert torch.equal(zb, ref_b)
        assert torch.equal(zs, ref_s)
        assert torch.equal(zb2, ref_b)
        zo = oracle_vcycle(lv, rs.cpu().numpy(), OracleOptions(max_levels=2), transpose=tr)
        assert _rel(zs.cpu().numpy(), zo) < tol


def test_noalloc_rejects_problems_beyond_the_scratch():
    from paper_1912_09056_amd.camg import CamgError

    # 60^3 over 61x61x60: about 1.39M unknowns, whose FP64 work vectors need
    # about 83 MB (the array holds 64 MiB)
    prob = make_contact_problem(3, (60, 60, 60), (61, 61, 60))
    s = _solver(prob, 0, max_levels=4)
    r = torch.from_numpy(np.random.default_rng(5).standard_normal(prob.n)).cuda()
    z = torch.zeros_like(r)
    with pytest.raises(CamgError) as e:
        s.vcycle_noalloc(r, z)
    assert e.value.code == -10
    assert torch.count_nonzero(z) == 0
    # the handle's own buffers are untouched: the regular V-cycle still works
    # and matches a fresh handle's
    z1 = s.vcycle(r)
    z2 = _solver(prob, 0, max_levels=4).vcycle(r)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
