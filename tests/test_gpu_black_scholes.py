"""Black-Scholes for_each (the paper's Black Scholes benchmark, section 5):
the GPU's binary32 call and put prices against the oracle's binary64
closed form on the same seeded options.

Bound: each price is S N(d1) - K e^{-rT} N(d2) (the put through parity);
the binary32 erfc / exp / log each err by a few ulp and the first-order
effect of an error in d1 cancels (S phi(d1) = K e^{-rT} phi(d2)), so the
absolute error stays within a small multiple of u32 (S + K); the tests use
32 u32 (S + K)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2406_00158_amd import binding as B
from paper_2406_00158_amd import inputs as I

from gpu_util import U32, announce, dev, dev_to_np, empty_like_segments, gather, place

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

BOUND = 32 * U32


def _check(t, lengths, call, put):
    wc, wp = O.black_scholes(*(I.split(t[n], lengths) for n in ("S", "K", "T", "V")), t["r"])
    wc, wp = np.concatenate(wc), np.concatenate(wp)
    scale = t["S"].astype(np.float64) + t["K"].astype(np.float64)
    ec, ep = np.abs(call.astype(np.float64) - wc) / scale, np.abs(put.astype(np.float64) - wp) / scale
    print(f"black-scholes: max |err| / (S + K) call {ec.max() / U32:.2f} u32, put {ep.max() / U32:.2f} u32")
    assert np.all(ec <= BOUND) and np.all(ep <= BOUND)


@pytest.mark.parametrize("lengths,layout", [([100_000], "separate"), ([4095, 4096, 4097, 1, 0, 8191], "carved"),
                                            ([0, 3, 0, 20000, 1, 33333], "separate"),
                                            ([(k * 37) % 1500 for k in range(130)], "carved")])
def test_black_scholes_prices(lengths, layout):
    announce("black-scholes", len(lengths), layout)
    n = sum(lengths)
    t = I.options(n=n, segments=1, seed=91)
    ins = [place(t[nm], lengths, layout) for nm in ("S", "K", "T", "V")]
    call = empty_like_segments(lengths, torch.float32)
    put = empty_like_segments(lengths, torch.float32)
    tab = B.segments(ins, [call, put])
    B.dr_for_each(tab, B.make_view("black_scholes", B.DR_F32, t["r"]), B.DR_F32)
    _check(t, lengths, gather(call), gather(put))


def test_black_scholes_rejects_other_algorithms_and_types():
    announce("black-scholes errors")
    x = torch.ones(10, device=dev())
    v = B.make_view("black_scholes", B.DR_F32, 0.02)
    with pytest.raises(B.DrError):
        B.dr_transform_reduce(B.segments([[x], [x], [x], [x]]), v, 0, 0.0, torch.zeros(1, dtype=torch.float64,
                                                                                         device=dev()))
    with pytest.raises(B.DrError):                       # one output only
        B.dr_for_each(B.segments([[x], [x], [x], [x]], [[x.clone()]]), v, B.DR_F32)
    xd = torch.ones(10, dtype=torch.float64, device=dev())
    with pytest.raises(B.DrError):
        B.dr_for_each(B.segments([[xd]] * 4, [[xd.clone()], [xd.clone()]]),
                      B.make_view("black_scholes", B.DR_F64, 0.02), B.DR_F64)
