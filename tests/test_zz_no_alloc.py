"""The allocation-free matvec (hbf_matvec_noalloc: fixed per-device scratch
instead of the context's workspace) gives the same products as hbf_matvec,
called twice in a row with the second input smaller, and rejects a product
whose scratch would exceed its fixed size."""
import math
import sys

import numpy as np
import pytest

from oracle import efie
from paper_1901_11371_amd import inputs

pytestmark = pytest.mark.gpu
KAPPA = 2 * math.pi


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_noalloc_matvec_equals_matvec(torch):
    from paper_1901_11371_amd._capi import HBF_EINVAL, HbfError
    from paper_1901_11371_amd.hbf import Context
    c1 = inputs.archimedean_spiral(4096)
    ctx1 = Context(c1, KAPPA, 64, 1e-6, dtype="c64", max_nrhs=128)
    rho, w = efie.segments(c1.xy, c1.node_off)
    A1 = efie.dense_A(rho, w, KAPPA)
    X = inputs.random_complex((6, 4096), 71)
    Xt = torch.tensor(X, dtype=torch.complex64, device="cuda")
    for adj in (False, True):
        _say(f"[noalloc] spiral 4096 c64, 6 RHS, adjoint={adj}")
        Y0 = ctx1.matvec(Xt, adjoint=adj).cpu().numpy()
        Y1 = ctx1.matvec_noalloc(Xt, adjoint=adj).cpu().numpy()
        ref = X @ (A1.conj() if adj else A1.T)
        _say(f"  vs matvec {_rel(Y1, Y0):.3e}, vs oracle {_rel(Y1, ref):.3e}")
        assert _rel(Y1, Y0) <= 1e-7
        assert _rel(Y1, ref) < 5e-6
    # second call, smaller input: another context (N = 2048, complex128), one RHS
    c2 = inputs.semicircle(2048)
    ctx2 = Context(c2, KAPPA, 64, 1e-6, dtype="c128", max_nrhs=1)
    rho2, w2 = efie.segments(c2.xy, c2.node_off)
    A2 = efie.dense_A(rho2, w2, KAPPA)
    x2 = inputs.random_complex(2048, 72)
    _say("[noalloc] semicircle 2048 c128, 1 RHS")
    y0 = ctx2.matvec(torch.tensor(x2, device="cuda")).cpu().numpy()
    y1 = ctx2.matvec_noalloc(torch.tensor(x2, device="cuda")).cpu().numpy()
    _say(f"  vs matvec {_rel(y1, y0):.3e}, vs oracle {_rel(y1, A2 @ x2):.3e}")
    assert _rel(y1, y0) <= 1e-12
    assert _rel(y1, A2 @ x2) < 5e-6
    # and the first context again with fewer right-hand sides (complex128 io)
    X2 = torch.tensor(X[:2], dtype=torch.complex128, device="cuda")
    Z0 = ctx1.matvec(X2).cpu().numpy()
    Z1 = ctx1.matvec_noalloc(X2).cpu().numpy()
    assert _rel(Z1, Z0) <= 1e-12
    assert _rel(Z1, X[:2] @ A1.T) < 5e-6
    # a product needing more than the fixed scratch is rejected
    big = torch.zeros((128, 4096), dtype=torch.complex128, device="cuda")
    with pytest.raises(HbfError) as e:
        ctx1.matvec_noalloc(big)
    assert e.value.status == HBF_EINVAL
    ctx1.close()
    ctx2.close()
