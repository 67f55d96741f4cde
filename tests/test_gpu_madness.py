"""GPU parity of the MADNESS separable contraction (dg_mra_apply, Sec. 7, Eq.
stock_mra) through the C ABI against the oracle's six-step evaluation.

Bars: FP64 1e-12 relative (per tensor, max norm over the batch), FP32 1e-5
(the chain multiplies six factors; each FP32 contraction of length <= 24
adds at most ~24 * 2^-24 relative to the sum of magnitudes, which for random
normal data is within a small factor of the result).  Sizes: tensor sizes
below, at and beyond one 16-wide MFMA tile, ranks 1..p, an empty and a
single-tensor batch.
"""
import sys

import numpy as np
import pytest

from oracle import madness

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(nb, p, q, seed):
    rng = np.random.default_rng(seed)
    S = rng.standard_normal((nb, p, p, p))
    ops = [rng.standard_normal(sh) / np.sqrt(sh[0]) for sh in ((p, q), (q, p)) * 3]
    return S, ops


def _rel(x, y):
    assert x.shape == y.shape
    if len(x) == 0:
        return 0.0
    d = np.abs(x - y).reshape(len(x), -1).max(axis=1)
    n = np.abs(y).reshape(len(y), -1).max(axis=1)
    return float(np.max(d / n))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nb,p,q", [(7, 5, 1), (33, 8, 3), (20, 16, 16), (9, 17, 5), (5, 20, 10), (3, 20, 20),
                                    (1, 12, 12), (0, 10, 4)])
def test_mra_against_oracle(nb, p, q, dtype):
    import paper_1903_11521_amd as dg
    _say(f"test_mra_against_oracle nb={nb} p={p} q={q} {dtype}")
    S, ops = _case(nb, p, q, 1000 + 37 * p + q)
    if dtype == torch.float32:
        S = S.astype(np.float32).astype(np.float64)
        ops = [o.astype(np.float32).astype(np.float64) for o in ops]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to("cuda:0")
    R = dg.mra_apply(dev(S), *[dev(o) for o in ops])
    torch.cuda.synchronize()
    got = R.double().cpu().numpy()
    ref = madness.apply(S, *ops)
    err = _rel(got, ref)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    _say("  max relative error %.3e (bar %.0e)" % (err, tol))
    assert err <= tol


def test_mra_fp32_largest():
    import paper_1903_11521_amd as dg
    S, ops = _case(4, 24, 12, 77)
    S = S.astype(np.float32).astype(np.float64)
    ops = [o.astype(np.float32).astype(np.float64) for o in ops]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(torch.float32).to("cuda:0")
    R = dg.mra_apply(dev(S), *[dev(o) for o in ops])
    torch.cuda.synchronize()
    assert _rel(R.double().cpu().numpy(), madness.apply(S, *ops)) <= 1e-5


def test_mra_refuses_unsupported():
    import paper_1903_11521_amd as dg
    z = lambda *sh: torch.zeros(sh, dtype=torch.float64, device="cuda:0")
    p, q = 21, 3
    with pytest.raises(dg.DGError, match="outside"):
        dg.mra_apply(z(1, p, p, p), z(p, q), z(q, p), z(p, q), z(q, p), z(p, q), z(q, p))
