"""GPU parity of the HIP hot path against the CPU FP64 oracle, through the
C ABI: matvec (forward and adjoint), the approximate-LU preconditioner in
both readings (forward and adjoint), complex64 and complex128 storage,
batched vs single right-hand sides, and argument checks."""
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


@pytest.fixture(scope="module")
def spiral(torch):
    c = inputs.archimedean_spiral(4096)
    rho, w = efie.segments(c.xy, c.node_off)
    return c, efie.dense_A(rho, w, KAPPA)


@pytest.fixture(scope="module")
def strip(torch):
    wl = inputs.workload(0)
    rho, w = efie.segments(wl.curves.xy, wl.curves.node_off)
    return wl.curves, efie.dense_A(rho, w, KAPPA)


def _ctx(c, dtype, prec="block", max_nrhs=8, z=None):
    from paper_1901_11371_amd.hbf import Context
    return Context(c, KAPPA, 64, 1e-6, dtype=dtype, prec=prec, max_nrhs=max_nrhs, z=z)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _rowmax(a, b):
    """Largest error of any single output row relative to the largest
    reference row (a per-row bar beside the relative L2 bar)."""
    a2 = np.atleast_2d(a)
    b2 = np.atleast_2d(b)
    return float(np.abs(a2 - b2).max() / np.abs(b2).max())


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("case", ["strip", "spiral"])
def test_matvec_matches_oracle(torch, strip, spiral, dtype, case):
    c, A = strip if case == "strip" else spiral
    _say(f"[matvec] case={case} dtype={dtype} N=4096")
    ctx = _ctx(c, dtype)
    x = inputs.random_complex(4096, 31)
    td = torch.complex64 if dtype == "c64" else torch.complex128
    y = ctx.matvec(torch.tensor(x, dtype=td, device="cuda")).cpu().numpy()
    torch.cuda.synchronize()
    err = _rel(y, A @ x)
    rowerr = _rowmax(y, A @ x)
    _say(f"  rel err {err:.3e} worst row {rowerr:.3e}")
    assert err < 5e-6 and rowerr < 2e-5
    ya = ctx.matvec(torch.tensor(x, dtype=td, device="cuda"), adjoint=True).cpu().numpy()
    erra = _rel(ya, A.conj().T @ x)
    _say(f"  adjoint rel err {erra:.3e}")
    assert erra < 5e-6
    ctx.close()


def test_matvec_batched_equals_single_and_fp64_io(torch, spiral):
    c, A = spiral
    _say("[matvec batched] spiral c64 R=5")
    ctx = _ctx(c, "c64")
    X = inputs.random_complex((5, 4096), 32)
    Xt = torch.tensor(X, dtype=torch.complex64, device="cuda")
    Y = ctx.matvec(Xt).cpu().numpy()
    for r in range(5):
        y1 = ctx.matvec(Xt[r].contiguous()).cpu().numpy()
        assert _rel(Y[r], y1) < 1e-6
    assert _rel(Y, X @ A.T) < 5e-6
    # complex128 io on the complex64 context: FP64 accumulation
    Y64 = ctx.matvec(torch.tensor(X, dtype=torch.complex128, device="cuda")).cpu().numpy()
    e64 = _rel(Y64, X @ A.T)
    _say(f"  c128-io rel err {e64:.3e}")
    assert e64 < 5e-6
    for adj in (False, True):
        Ya = ctx.matvec(Xt, adjoint=adj).cpu().numpy()
        ref = X @ (A.conj() if adj else A.T)
        assert _rel(Ya, ref) < 5e-6
    ctx.close()


@pytest.mark.parametrize("prec", ["block", "paper"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_precond_matches_oracle(torch, spiral, prec, dtype):
    c, A = spiral
    _say(f"[precond] prec={prec} dtype={dtype}")
    ctx = _ctx(c, dtype, prec=prec)
    td = torch.complex64 if dtype == "c64" else torch.complex128
    R = inputs.random_complex((3, 4096), 33)
    f = (lambda v, adj: efie.precond_block_apply(A, v, 64, adjoint=adj)) if prec == "block" else \
        (lambda v, adj: efie.precond_paper_apply(A, v, adjoint=adj))
    for adj in (False, True):
        Z = ctx.precond(torch.tensor(R, dtype=td, device="cuda"), adjoint=adj).cpu().numpy()
        ref = np.stack([f(R[i], adj) for i in range(3)])
        err = _rel(Z, ref)
        rowerr = _rowmax(Z, ref)
        _say(f"  adjoint={adj} rel err {err:.3e} worst row {rowerr:.3e}")
        assert err < (2e-6 if dtype == "c128" else 5e-5)
        assert rowerr < (1e-5 if dtype == "c128" else 2e-4)
        z1 = ctx.precond(torch.tensor(R[1], dtype=td, device="cuda"), adjoint=adj).cpu().numpy()
        assert _rel(z1, Z[1]) < (1e-12 if dtype == "c128" else 1e-5)
    ctx.close()


TUNINGS = [
    {"prog_levels": 0},
    {"prog_levels": 2},
    {"prog_levels": 3, "lane_split": 0},
    {"prog_levels": 12},
    {"prog_pipe": 0},
    {"pipe_max_r": 0, "wave_units": 1},
    {"pipe_max_r": 0, "wave_units": 0},
    {"use_graphs": 0, "prog_levels": 4},
    {"sweep_rc1": 1},
    {"pipe_max_r": 0, "wave_units": 1, "sweep_rc1": 1},
    {"pipe_max_r": 8, "sweep_pipe_max_r": 8},
    {"prog_lds": 0},
    {"prog_lds": 0, "prog_levels": 6},
    {"mv_direct": 0},
    {"mv_direct": 0, "lane_split": 0},
    {"lane_units": 0},
    {"lane_units": 0, "lane_split": 0},
    {"lane_max_entries": 128},
    {"lane_max_entries": 1 << 20},
    {"lane_scatter_split": 0},
    {"lane_scatter_split": 0, "lane_max_entries": 1 << 20},
    {"prog_levels": 7},
    {"r1_max_blocks": 2048},
    {"r1_max_blocks": 3, "sweep_pipe_max_r": 8},
    {"mfma_min_r": 1},
    {"mfma_min_r": 1, "mv_direct": 0},
    {"mfma_min_r": 1, "prog_levels": 0},
    {"mfma_min_r": 1, "prog_levels": 3, "use_graphs": 0},
    {"mfma_min_r": 1, "mfma_tiles": 1},
    {"mfma_min_r": 1, "mfma_tiles": 2, "mv_direct": 0},
    {"mfma_min_r": 1, "mfma_split_rows": 0},
]


@pytest.fixture(scope="module")
def tuning_refs(spiral):
    """Oracle matvec and preconditioner of the five seeded RHS the tuning
    tests share (forward and adjoint), computed once."""
    c, A = spiral
    R = inputs.random_complex((5, 4096), 35)
    refs = {}
    for adj in (False, True):
        ref = ((A.conj().T if adj else A) @ R.T).T
        refz = np.stack([efie.precond_block_apply(A, R[i], 64, adjoint=adj) for i in range(5)])
        refs[adj] = (ref, refz)
    return R, refs


@pytest.mark.parametrize("tuning", TUNINGS, ids=lambda t: ",".join(f"{k}={v}" for k, v in t.items()))
def test_execution_parameters_keep_results(torch, spiral, tuning_refs, tuning):
    """Every execution parameter the autotuner may pick gives the oracle's
    matvec and preconditioner (forward and adjoint, 1 and 5 RHS)."""
    c, A = spiral
    R, refs = tuning_refs
    _say(f"[tuning] {tuning}")
    ctx = _ctx(c, "c64")
    for k, v in tuning.items():
        ctx.tune(k, v)
    Rt = torch.tensor(R, dtype=torch.complex64, device="cuda")
    for adj in (False, True):
        ref, refz = refs[adj]
        Y = ctx.matvec(Rt, adjoint=adj).cpu().numpy()
        err = _rel(Y, ref)
        y1 = ctx.matvec(Rt[2].contiguous(), adjoint=adj).cpu().numpy()
        _say(f"  matvec adjoint={adj} rel err {err:.3e}")
        assert err < 5e-6 and _rel(y1, Y[2]) < 1e-5
        Z = ctx.precond(Rt, adjoint=adj).cpu().numpy()
        errz = _rel(Z, refz)
        z1 = ctx.precond(Rt[2].contiguous(), adjoint=adj).cpu().numpy()
        _say(f"  precond adjoint={adj} rel err {errz:.3e}")
        assert errz < 5e-5 and _rel(z1, Z[2]) < 1e-5
    ctx.close()


@pytest.fixture(scope="module")
def refs64(spiral):
    """Oracle products of the 64 seeded RHS of the matrix-core tests (A X,
    A^H X, and P^-1, P^-H of the first 16), computed once: the oracle's
    block substitutions take all 16 columns in one dense solve each."""
    c, A = spiral
    X = inputs.random_complex((64, 4096), 37)
    out = {"X": X}
    for adj in (False, True):
        out[("mv", adj)] = X @ (A.conj() if adj else A.T)
        out[("pc", adj)] = efie.precond_block_apply(A, X[:16].T, 64, adjoint=adj).T
    return out


@pytest.mark.parametrize("mfma,tiles", [(1, 4), (1, 2), (1, 1), (0, 4)])
def test_64_rhs_on_matrix_cores(torch, spiral, refs64, mfma, tiles):
    """64 right-hand sides (the batched launch shape): matvec and
    preconditioner, forward and adjoint, with the matrix-core stage launches
    (and without them), against the oracle, with relative L2 and worst-row
    bars, and each batch column against the single-RHS product."""
    c, A = spiral
    _say(f"[64 rhs] spiral 4096 c64 mfma={mfma} tiles={tiles}")
    ctx = _ctx(c, "c64", max_nrhs=64)
    ctx.tune("mfma", mfma)
    ctx.tune("mfma_tiles", tiles)
    X = refs64["X"]
    Xt = torch.tensor(X, dtype=torch.complex64, device="cuda")
    for adj in (False, True):
        Y = ctx.matvec(Xt, adjoint=adj).cpu().numpy()
        ref = refs64[("mv", adj)]
        err, rowerr = _rel(Y, ref), _rowmax(Y, ref)
        y1 = ctx.matvec(Xt[40].contiguous(), adjoint=adj).cpu().numpy()
        _say(f"  matvec adjoint={adj} rel err {err:.3e} worst row {rowerr:.3e} col40 vs single {_rel(Y[40], y1):.2e}")
        assert err < 5e-6 and rowerr < 2e-5 and _rel(Y[40], y1) < 1e-5
        Z = ctx.precond(Xt[:16].contiguous(), adjoint=adj).cpu().numpy()
        refz = refs64[("pc", adj)]
        errz, rowz = _rel(Z, refz), _rowmax(Z, refz)
        _say(f"  precond (16 rhs) adjoint={adj} rel err {errz:.3e} worst row {rowz:.3e}")
        assert errz < 5e-5 and rowz < 2e-4
    ctx.close()


@pytest.mark.parametrize("superleaf", [3])
@pytest.mark.parametrize("prec", ["block", "paper"])
def test_superleaf_sizes(torch, spiral, prec, superleaf):
    """The leaf solves of the sweeps invert diagonal blocks of 2^superleaf
    leaves; the 8-leaf size gives the oracle's preconditioner as the default
    4-leaf one does (1, 5 and 16 RHS, forward and adjoint)."""
    from paper_1901_11371_amd.hbf import Context
    c, A = spiral
    _say(f"[superleaf] {superleaf} prec={prec}")
    ctx = Context(c, KAPPA, 64, 1e-6, dtype="c64", prec=prec, max_nrhs=16, superleaf=superleaf)
    X = inputs.random_complex((16, 4096), 38)
    f = (lambda v, adj: efie.precond_block_apply(A, v, 64, adjoint=adj)) if prec == "block" else \
        (lambda v, adj: efie.precond_paper_apply(A, v, adjoint=adj))
    for adj in (False, True):
        ref = f(X.T, adj).T
        for nr in (1, 5, 16):
            Xt = torch.tensor(X[:nr], dtype=torch.complex64, device="cuda")
            Z = ctx.precond(Xt if nr > 1 else Xt[0], adjoint=adj).cpu().numpy().reshape(nr, -1)
            err, rowerr = _rel(Z, ref[:nr]), _rowmax(Z, ref[:nr])
            _say(f"  adjoint={adj} nrhs={nr} rel err {err:.3e} worst row {rowerr:.3e}")
            assert err < 5e-5 and rowerr < 2e-4
    ctx.close()


def test_bitwise_determinism(torch, spiral):
    """No kernel uses atomics for results and every reduction has a fixed
    order: repeated products and solves are bit-identical (1 and 64 RHS,
    forward and adjoint, the matrix-core and the pipelined launches)."""
    c, _ = spiral
    ctx = _ctx(c, "c64", max_nrhs=64)
    X = torch.tensor(inputs.random_complex((64, 4096), 39), dtype=torch.complex64, device="cuda")
    for Xi in (X, X[5].contiguous()):
        for adj in (False, True):
            a1 = ctx.matvec(Xi, adjoint=adj).cpu().numpy()
            a2 = ctx.matvec(Xi, adjoint=adj).cpu().numpy()
            p1 = ctx.precond(Xi, adjoint=adj).cpu().numpy()
            p2 = ctx.precond(Xi, adjoint=adj).cpu().numpy()
            assert np.array_equal(a1, a2) and np.array_equal(p1, p2)
    B = torch.tensor(inputs.plane_wave_rhs(c, inputs.uniform_angles(3)), device="cuda")
    x1, i1, _ = ctx.solve(B, tol=1e-6, max_iters=60)
    x2, i2, _ = ctx.solve(B, tol=1e-6, max_iters=60)
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy()) and i1 == i2
    ctx.close()


def test_nrhs_beyond_max_is_rejected(torch, spiral):
    from paper_1901_11371_amd._capi import HBF_EINVAL, HbfError
    c, _ = spiral
    ctx = _ctx(c, "c64", max_nrhs=2)
    x = torch.zeros((3, 4096), dtype=torch.complex64, device="cuda")
    with pytest.raises(HbfError) as e:
        ctx.matvec(x)
    assert e.value.status == HBF_EINVAL
    with pytest.raises(HbfError) as e:
        ctx.precond(x)
    assert e.value.status == HBF_EINVAL
    ctx.close()


def test_impedance_and_refactor(torch):
    _say("[impedance] semicircle 2048")
    c = inputs.semicircle(2048)
    rho, w = efie.segments(c.xy, c.node_off)
    z = inputs.impedance(2048, 7)
    ctx = _ctx(c, "c128")
    ctx.set_impedance(z)
    A = efie.dense_A(rho, w, KAPPA, z=z)
    x = inputs.random_complex(2048, 34)
    y = ctx.matvec(torch.tensor(x, device="cuda")).cpu().numpy()
    assert _rel(y, A @ x) < 5e-6
    zz = ctx.precond(torch.tensor(x, device="cuda")).cpu().numpy()
    assert _rel(zz, efie.precond_block_apply(A, x, 64)) < 2e-6
    ctx.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_any_size_matches_oracle(torch, dtype):
    """N = 2049 on the spiral: not n0 2^V, leaves at two depths of the
    bisection, padded to 4096 inside the library.  Matvec and preconditioner
    (forward, adjoint; 1 and 3 right-hand sides), the allocation-free matvec,
    an impedance set after construction, and the impedance gradient's
    length, against the dense oracle."""
    n = 2049
    _say(f"[any N] spiral N={n} dtype={dtype}")
    c = inputs.archimedean_spiral(n)
    rho, w = efie.segments(c.xy, c.node_off)
    A = efie.dense_A(rho, w, KAPPA)
    ctx = _ctx(c, dtype)
    assert ctx.n == n and ctx.stats["n_internal"] == 4096
    td = torch.complex64 if dtype == "c64" else torch.complex128
    X = inputs.random_complex((3, n), 45)
    for adj in (False, True):
        Ae = A.conj().T if adj else A
        for xs in (X[0], X):
            y = ctx.matvec(torch.tensor(xs, dtype=td, device="cuda"), adjoint=adj).cpu().numpy()
            ref = (Ae @ xs.T).T
            assert _rel(y, ref) < 5e-6 and _rowmax(y, ref) < 2e-5, (adj, xs.ndim)
            zp = ctx.precond(torch.tensor(xs, dtype=td, device="cuda"), adjoint=adj).cpu().numpy()
            zr = np.stack([efie.precond_block_apply(A, v, 64, adjoint=adj) for v in np.atleast_2d(xs)])
            assert _rel(np.atleast_2d(zp), zr) < 5e-6, (adj, xs.ndim)
    y1 = ctx.matvec(torch.tensor(X[0], dtype=td, device="cuda")).cpu().numpy()
    y2 = ctx.matvec_noalloc(torch.tensor(X[0], dtype=td, device="cuda")).cpu().numpy()
    assert np.array_equal(y1, y2)
    z = inputs.impedance(n, 8)
    ctx.set_impedance(z)
    Az = efie.dense_A(rho, w, KAPPA, z=z)
    y = ctx.matvec(torch.tensor(X, dtype=td, device="cuda")).cpu().numpy()
    assert _rel(y, (Az @ X.T).T) < 5e-6
    g = ctx.impedance_grad(torch.tensor(X, dtype=td, device="cuda"), torch.tensor(X, dtype=td, device="cuda"))
    assert g.shape == (n,)
    ref = -np.sum(X * np.conj(X), axis=0)
    assert _rel(g.cpu().numpy(), ref) < 1e-6
    with pytest.raises(ValueError):
        ctx.set_impedance(np.zeros(4096))
    ctx.close()


def test_any_size_solve_matches_dense_lu(torch):
    """Batched complex64 solve with FP64 refinement at N = 1000 (padded to
    1024), 3 plane waves, GMRES and TFQMR, against dense LU."""
    from paper_1901_11371_amd.hbf import Context
    n = 1000
    _say(f"[any N] semicircle N={n} solve")
    c = inputs.semicircle(n)
    rho, w = efie.segments(c.xy, c.node_off)
    A = efie.dense_A(rho, w, KAPPA)
    B = inputs.plane_wave_rhs(c, inputs.uniform_angles(3))
    Xr = efie.lu_solve(A, B.T).T
    ctx = Context(c, KAPPA, 64, 1e-6, dtype="c64", max_nrhs=4)
    for method in ("gmres", "tfqmr"):
        X, info, st = ctx.solve(torch.tensor(B, device="cuda"), tol=1e-7, max_iters=300, method=method)
        X = X.cpu().numpy()
        errs = [_rel(X[r], Xr[r]) for r in range(3)]
        _say(f"  {method}: errs max {max(errs):.2e} iters {[i['iters'] for i in info]}")
        assert st == 0 and all(i["converged"] for i in info)
        assert max(errs) < 1e-5
    ctx.close()


def test_singular_leaf_and_allocation_failure_are_reported(torch):
    """A leaf whose paper-reading upper factor has an exact zero on its
    diagonal (impedance z_i = -Z_ii, taken from the library's own entries) is
    reported as HBF_ESINGULAR by hbf_build and by hbf_set_impedance; a
    workspace beyond the device memory is reported as HBF_ENOMEM."""
    from paper_1901_11371_amd._capi import HBF_ENOMEM, HBF_ESINGULAR, HbfError
    from paper_1901_11371_amd.hbf import Context, HostPlan
    n = 1024
    c = inputs.archimedean_spiral(n)
    plan = HostPlan(c, KAPPA, 64, 1e-6, prec="paper")
    i = 70
    zii = plan.entries(np.array([i]), np.array([i]))[0, 0]
    z = np.zeros(n, dtype=np.complex128)
    z[i] = -zii
    _say("[errors] singular leaf at build")
    with pytest.raises(HbfError) as e:
        Context(c, KAPPA, 64, 1e-6, dtype="c64", prec="paper", z=z)
    assert e.value.status == HBF_ESINGULAR
    _say("[errors] singular leaf at set_impedance")
    ctx = Context(c, KAPPA, 64, 1e-6, dtype="c64", prec="paper")
    with pytest.raises(HbfError) as e:
        ctx.set_impedance(z)
    assert e.value.status == HBF_ESINGULAR
    # a valid impedance makes the context usable again
    ctx.set_impedance(np.zeros(n, dtype=np.complex128))
    rho, w = efie.segments(c.xy, c.node_off)
    A = efie.dense_A(rho, w, KAPPA)
    x = inputs.random_complex(n, 36)
    zz = ctx.precond(torch.tensor(x, dtype=torch.complex64, device="cuda")).cpu().numpy()
    assert _rel(zz, efie.precond_paper_apply(A, x)) < 5e-5
    ctx.close()
    _say("[errors] workspace beyond device memory")
    with pytest.raises(HbfError) as e:
        Context(c, KAPPA, 64, 1e-6, dtype="c64", max_nrhs=1 << 24)
    assert e.value.status == HBF_ENOMEM
