"""GPU parity of the Cauchy-like product (Sec. 6.3, eqs. (6.1)-(6.2)) through
the C ABI: smash_matvec_cauchy_like against the FP64 oracle's product by
(6.2) over its own HSS approximation (same tree, skeletons and generators as
the GPU's, so within 1e-10 relative Frobenius with FP64 apply, 1e-5 with
FP32 apply on FP32-rounded inputs), against the sum of plain products of the
same handle, and against the dense definition (6.1) within the construction's
accuracy."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1705_05443_amd import api  # noqa: E402
from paper_1705_05443_amd import workloads as W  # noqa: E402

KW = dict(kernel="cauchy", leaf=50, order=16, adm="weak", tol=1e-8, eps_svd=1e-9, tau=0.6)
POINTS = {
    "chebyshev_pair": lambda n: W.chebyshev_pair(n, 1),
    "interlaced_6_3": lambda n: W.interlaced_pair(n, 1),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("pts", list(POINTS))
def test_cauchy_like_fp64_parity(pts, p):
    n = 3000
    x, y = POINTS[pts](n)
    w, v = W.cauchy_like_generators(n, n, p, seed=2)
    q = W.rhs(n, 3, seed=3)
    print("case", pts, "p", p, flush=True)
    o = O.Oracle(x, y, kernel="cauchy", leaf=50, order=16, adm=0, tol=1e-8, eps_svd=1e-9, tau=0.6)
    g = api.Smash(dev(x), dev(y), **KW)
    z = g.matvec_cauchy_like(dev(q), dev(w), dev(v)).cpu().numpy()
    zo = o.cauchy_like_matvec(w, v, q)
    assert relerr(z, zo) < 1e-10
    assert relerr(z, O.cauchy_like_dense(x, y, w, v, q)) < 1e-8
    # the same as the weighted sum of the handle's plain products
    zs = sum(w[:, l:l + 1] * g.matvec(dev(v[:, l:l + 1] * q)).cpu().numpy() for l in range(p))
    assert relerr(z, zs) < 1e-12
    g.close()


def test_cauchy_like_fp32_apply():
    n = 3000
    x, y = W.chebyshev_pair(n, 1)
    w, v = W.cauchy_like_generators(n, n, 2, seed=4)
    q = W.rhs(n, 5, seed=5).astype(np.float32)
    o = O.Oracle(x, y, kernel="cauchy", leaf=50, order=16, adm=0, tol=1e-8, eps_svd=1e-9, tau=0.6)
    g = api.Smash(dev(x), dev(y), apply_prec="f32", **KW)
    z = g.matvec_cauchy_like(dev(q), dev(w), dev(v)).cpu().numpy()
    assert relerr(z, o.cauchy_like_matvec(w, v, q.astype(np.float64))) < 1e-5
    g.close()


def test_cauchy_like_argument_errors():
    n = 500
    x, y = W.chebyshev_pair(n, 1)
    g = api.Smash(dev(x), dev(y), **KW)
    q = dev(W.rhs(n, 2, seed=1))
    w, v = W.cauchy_like_generators(n, n, 2, seed=1)
    with pytest.raises(TypeError):
        g.matvec_cauchy_like(q, dev(w).float(), dev(v))
    with pytest.raises(ValueError):
        g.matvec_cauchy_like(q, dev(w), dev(v[:, :1]))
    big = np.ones((n, 17))
    with pytest.raises(api.SmashError):
        g.matvec_cauchy_like(q, dev(big), dev(big))
    # the handle stays usable after a rejected call
    z = g.matvec_cauchy_like(q, dev(w), dev(v)).cpu().numpy()
    assert np.isfinite(z).all()
    g.close()


@pytest.mark.parametrize("basis", ["chebyshev", "taylor"])
def test_cauchy_like_distinct_counts_max_p_and_vector(basis):
    """nx != ny, the largest generator count (SMASH_CAUCHY_LIKE_MAX_P = 16), a
    single right-hand side passed as a vector, and the Taylor basis
    (eqs. (2.4)-(2.5)) under the Cauchy matrix: still within 1e-10 of the
    oracle's (6.2) product and within the construction's accuracy of (6.1)."""
    nx, ny, p = 2000, 2600, 16
    rng = np.random.default_rng(31)
    x = np.sort(rng.random(nx))[:, None]
    y = np.sort(rng.random(ny))[:, None] + 0.5 / ny
    w, v = W.cauchy_like_generators(nx, ny, p, seed=8)
    q = W.rhs(ny, 1, seed=9)[:, 0]
    kw = dict(KW, basis=basis)
    o = O.Oracle(x, y, kernel="cauchy", leaf=50, order=16, adm=0, tol=1e-8, eps_svd=1e-9,
                 tau=0.6, basis=basis)
    g = api.Smash(dev(x), dev(y), **kw)
    z = g.matvec_cauchy_like(dev(q), dev(w), dev(v)).cpu().numpy()
    assert z.shape == (nx,)
    assert relerr(z, o.cauchy_like_matvec(w, v, q)) < 1e-10
    assert relerr(z, O.cauchy_like_dense(x, y, w, v, q)) < 1e-7
    g.close()
