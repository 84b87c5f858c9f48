"""Backward passes: torch.autograd.gradcheck (central finite differences) on
64-element binary64 cases with several segmentations, closed forms of the
adjoints, and binary32 gradients against the binary64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2406_00158_amd import autograd as AG
from paper_2406_00158_amd import inputs as I

from gpu_util import announce, dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

# 64 elements in total: several small batches (the finite-difference cases)
SEGS64 = [[64], [1, 7, 56], [32, 32], [0, 5, 0, 59], [13, 1, 1, 20, 29]]


def _rand64(seed, n=64):
    g = np.random.default_rng(seed)
    return torch.from_numpy(g.standard_normal(n)).to(dev()).requires_grad_(True)


@pytest.mark.parametrize("lengths", SEGS64)
@pytest.mark.parametrize("mode", ["concat", "batch"])
def test_gradcheck_scan(lengths, mode):
    announce("gradcheck scan", lengths, mode)
    x = _rand64(1)
    assert torch.autograd.gradcheck(lambda t: AG.inclusive_scan(t, lengths, mode), (x,), eps=1e-6, atol=1e-8)


@pytest.mark.parametrize("lengths", SEGS64)
@pytest.mark.parametrize("mode", ["concat", "batch"])
def test_gradcheck_dot_and_sumsq(lengths, mode):
    announce("gradcheck dot", lengths, mode)
    x, y = _rand64(2), _rand64(3)
    assert torch.autograd.gradcheck(lambda a, b: AG.dot(a, b, lengths, mode), (x, y), eps=1e-6, atol=1e-8)
    assert torch.autograd.gradcheck(lambda a: AG.sum_of_squares(a, lengths, mode), (x,), eps=1e-6, atol=1e-8)


@pytest.mark.parametrize("lengths", SEGS64)
@pytest.mark.parametrize("mode", ["concat", "batch"])
def test_gradcheck_fused_scan_dot(lengths, mode):
    announce("gradcheck scan_dot", lengths, mode)
    x, y = _rand64(4), _rand64(5)
    assert torch.autograd.gradcheck(lambda a, b: AG.scan_dot(a, b, lengths, mode), (x, y), eps=1e-6, atol=1e-8)


def test_scan_adjoint_of_ones_closed_form():
    # d/dx_i of sum(scan(x)) = number of positions at or after i (in its range)
    lengths = [5000, 1, 0, 70000, 4096]
    n = sum(lengths)
    announce("scan adjoint ones")
    for mode in ("concat", "batch"):
        x = torch.zeros(n, device=dev(), requires_grad=True)
        AG.inclusive_scan(x, lengths, mode).sum().backward()
        if mode == "concat":
            want = np.arange(n, 0, -1, dtype=np.float32)
        else:
            want = np.concatenate([np.arange(L, 0, -1, dtype=np.float32) for L in lengths])
        assert np.array_equal(x.grad.cpu().numpy(), want)


def test_dot_gradient_with_unit_upstream_is_exact():
    lengths = I.lengths_loguniform(200, 4096, 1 << 18, 3)
    n = sum(lengths)
    announce("dot grad exact")
    x = torch.from_numpy(I.normal_f32(n, 7)).to(dev()).requires_grad_(True)
    y = torch.from_numpy(I.normal_f32(n, 8)).to(dev()).requires_grad_(True)
    AG.dot(x, y, lengths, "batch").sum().backward()
    assert torch.equal(x.grad, y.detach()) and torch.equal(y.grad, x.detach())


def test_fp32_backward_matches_fp64_oracle():
    lengths = I.lengths_loguniform(300, 1 << 14, 1 << 21, 11)
    n = sum(lengths)
    announce("fp32 backward vs oracle", n)
    xs, ys = I.normal_f32(n, 12), I.normal_f32(n, 13)
    x = torch.from_numpy(xs).to(dev()).requires_grad_(True)
    y = torch.from_numpy(ys).to(dev()).requires_grad_(True)
    s, d = AG.scan_dot(x, y, lengths, "batch")
    gsn = I.normal_f32(n, 14)
    gdn = I.normal_f32(len(lengths), 15).astype(np.float64)
    torch.autograd.backward([s, d], [torch.from_numpy(gsn).to(dev()), torch.from_numpy(gdn).to(dev())])
    # oracle: gx = reverse scan(g_s) + g_d * y ; gy = g_d * x  (binary64)
    rs = np.concatenate(O.scan(I.split(gsn, lengths), None, O.F32, O.IDENTITY, mode=O.BATCH, reverse=True))
    gdx = np.concatenate(O.reduce_grad(I.split(xs, lengths), I.split(ys, lengths), O.F32, O.MUL, gdn, 0,
                                       mode=O.BATCH))
    gdy = np.concatenate(O.reduce_grad(I.split(xs, lengths), I.split(ys, lengths), O.F32, O.MUL, gdn, 1,
                                       mode=O.BATCH))
    _, absr = O.scan(I.split(gsn, lengths), None, O.F32, O.IDENTITY, mode=O.BATCH, reverse=True, want_abs=True)
    absr = np.concatenate(absr)
    gx = x.grad.cpu().numpy().astype(np.float64)
    u = 2.0 ** -24
    # reverse scan in binary32 tiles + binary64 carries, one rounding of g*y, one add
    bound = 26 * u * absr + 2 * u * (np.abs(rs) + np.abs(gdx)) + u * np.abs(gdx)
    assert np.all(np.abs(gx - (rs + gdx)) <= bound)
    assert np.array_equal(y.grad.cpu().numpy(), gdy.astype(np.float32))
