"""smash_matvec_noalloc (vectors in the library's per-device array, no
allocation) against smash_matvec through the C ABI: the same products, bit
for bit, on two calls in a row where the second has a smaller input (fewer
points and right-hand sides, so the array still holds the first call's
values beyond the second's vectors), in each apply precision, with more
right-hand sides than one pass holds, and a handle too large for the array
rejected with the sizes named."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1705_05443_amd import api  # noqa: E402
from paper_1705_05443_amd import workloads as W  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


KW = dict(kernel="log_r", leaf=64, order=8, adm="strong", tol=1e-8, tau=0.7,
          root=((0.0, 0.0), 1.0))


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_noalloc_equals_allocating_product(prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    ev = "f64" if prec == "f64" else "f32"
    big = api.Smash(dev(W.uniform(20000, 2, 61)), apply_prec=prec, eval_prec=ev, **KW)
    small = api.Smash(dev(W.uniform(3000, 2, 62)), apply_prec=prec, eval_prec=ev, **KW)
    for h, nrhs in ((big, 40), (small, 5), (big, 130), (small, 1)):
        print("noalloc", prec, h.nx, nrhs, flush=True)
        X = dev(W.rhs(h.ny, nrhs, seed=nrhs)).to(dt)
        ref = h.matvec(X)
        out = torch.full_like(ref, float("nan"))
        h.matvec_noalloc(X, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (prec, h.nx, nrhs)
    big.close()
    small.close()


def test_noalloc_fp64_matches_oracle_and_strided_input():
    x = W.uniform(5000, 2, 63)
    o = O.Oracle(x, None, kernel="log_r", leaf=64, order=8, adm=1, tol=1e-8, tau=0.7,
                 root=((0.0, 0.0), 1.0))
    h = api.Smash(dev(x), **KW)
    q = W.rhs(5000, 24, seed=64)
    Q = dev(q)
    z = h.matvec_noalloc(Q[:, 3:20]).cpu().numpy()
    zo = o.matvec(q[:, 3:20])
    assert np.linalg.norm(z - zo) / np.linalg.norm(zo) < 1e-10
    h.close()


def test_noalloc_rejects_a_handle_beyond_the_array():
    # 2^20 slot rows of FP64 at 16 columns need 128 MiB, twice the array
    x = W.uniform(1 << 20, 1, 65)
    h = api.Smash(dev(x), kernel="inv_r", leaf=64, order=4, adm="strong", tol=1e-6, tau=0.6,
                  root=((0.0,), 1.0))
    X = torch.zeros((h.ny, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(api.SmashError) as e:
        h.matvec_noalloc(X)
    assert e.value.code == -1 and "no-allocation" in str(e.value)
    h.close()
