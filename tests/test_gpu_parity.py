"""GPU parity: the HIP library against the FP64 CPU oracle, through the C ABI.

Integer outputs (permutation, tree, pair lists, near sets, ranks, skeleton
sets) must be bit-exact.  FP64 construction: H^2 interpolative-decomposition
coefficients G within 1e-10 of the oracle's (relative to max(1, |G|) per node,
or within the forward-error bound of the node's skeleton conditioning;
HSS G by the properties in _check_hss_ids) and products within 1e-10
relative Frobenius.  FP32 apply: within
1e-5 relative Frobenius of the oracle's FP64 product on the FP32-rounded
right-hand sides.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1705_05443_amd import api  # noqa: E402
from paper_1705_05443_amd import workloads as W  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = {
    # name: (points(), kwargs)
    "hss1d_small": (lambda: (W.uniform(700, 1, 3), None),
                    dict(kernel="inv_r", leaf=16, order=8, adm="weak", tol=1e-9, eps_svd=1e-9,
                         tau=0.6, root=((0.0,), 1.0))),
    "hss1d_cfg": (lambda: W.points(W.CONFIGS["hss1d_inv_r_2048"]),
                  dict(kernel="inv_r", leaf=32, order=10, adm="weak", tol=1e-10, eps_svd=1e-10,
                       tau=0.6, root=((0.0,), 1.0))),
    "h2_2d_log": (lambda: (W.uniform(5000, 2, 5), None),
                  dict(kernel="log_r", leaf=64, order=8, adm="strong", tol=1e-8, tau=0.7,
                       root=((0.0, 0.0), 1.0))),
    "h2_3d_clusters": (lambda: (W.clusters(6000, 3, 6), None),
                       dict(kernel="inv_r", leaf=128, order=5, adm="strong", tol=1e-6, tau=0.7,
                            root=((0.0, 0.0, 0.0), 1.0))),
    # c = 64 with parent grids of up to 512 points: a level splits between
    # the register form (grids <= 256) and the wide form (the larger ones)
    "h2_3d_p4_split": (lambda: (W.clusters(9000, 3, 9), None),
                       dict(kernel="inv_r", leaf=128, order=4, adm="strong", tol=1e-7, tau=0.7,
                            root=((0.0, 0.0, 0.0), 1.0))),
    # swap bound f close to 1: Gu-Eisenstat swaps in many nodes, whose grids
    # (up to 8 x 125 points) split over several workgroups in k_compr_dq
    "h2_3d_swaps": (lambda: (W.clusters(6000, 3, 12), None),
                    dict(kernel="inv_r", leaf=128, order=5, adm="strong", tol=1e-6, tau=0.7,
                         f=1.05, root=((0.0, 0.0, 0.0), 1.0))),
    "h2_1d_exp": (lambda: (W.uniform(3000, 1, 8), None),
                  dict(kernel="exp_r", leaf=40, order=9, adm="strong", tol=1e-10, tau=0.6)),
    "hss_cauchy_xy": (lambda: W.chebyshev_pair(3000, 4),
                      dict(kernel="cauchy", leaf=64, order=16, adm="weak", tol=1e-8,
                           eps_svd=1e-9, tau=0.6)),
    # the Taylor basis of eqs. (2.4)-(2.5) in place of interpolation
    "hss_cauchy_taylor": (lambda: W.chebyshev_pair(3000, 4),
                          dict(kernel="cauchy", leaf=64, order=16, adm="weak", tol=1e-8,
                               eps_svd=1e-9, tau=0.6, basis="taylor")),
    "h2_1d_inv_r_taylor": (lambda: (W.uniform(3000, 1, 11), None),
                           dict(kernel="inv_r", leaf=40, order=12, adm="strong", tol=1e-10,
                                tau=0.6, root=((0.0,), 1.0), basis="taylor")),
    # Laplace double layer on the curves of Sec. 6.4 (Nystrom data as point data)
    "hss_dl_ram_head": (lambda: (W.curve("ram_head", 1280)[0], None),
                        dict(kernel="double_layer", leaf=50, order=5, adm="weak", tol=1e-10,
                             eps_svd=1e-11, tau=0.6,
                             point_data=W.curve("ram_head", 1280)[1])),
    "hss_dl_sunflower": (lambda: (W.curve("sunflower", 640)[0], None),
                         dict(kernel="double_layer", leaf=50, order=5, adm="weak", tol=1e-10,
                              eps_svd=1e-11, tau=0.6,
                              point_data=W.curve("sunflower", 640)[1])),
}
DL = {k for k, v in CASES.items() if v[1]["kernel"] == "double_layer"}


def _oracle_kwargs(kw):
    ok = dict(kw)
    ok["adm"] = api.ADM[kw["adm"]]
    return ok


def _gpu_kwargs(kw):
    gk = dict(kw)
    if gk.get("point_data") is not None:
        gk["point_data"] = dev(gk["point_data"])
    return gk


_cache = {}


def pair_for(name):
    if name not in _cache:
        mk, kw = CASES[name]
        x, y = mk()
        o = O.Oracle(x, y, **_oracle_kwargs(kw))
        g = api.Smash(dev(x), None if y is None else dev(y), **_gpu_kwargs(kw))
        _cache[name] = (x, y, o, g)
    return _cache[name]


def test_swap_case_swaps_in_split_grids():
    """The f = 1.05 case exercises the swap path of the register-resident
    compr: swaps happen, and some grids exceed one workgroup's 128 columns
    (its skeletons and G are checked against the oracle by the tests
    parametrized over the cases)."""
    x, y, o, g = pair_for("h2_3d_swaps")
    inf = g.info()
    m = g.export("ranks").reshape(-1, 6)[:, 0]
    print("swaps", inf["total_swaps"], "largest grid", int(m.max()), flush=True)
    assert inf["total_swaps"] > 0
    assert m.max() > 128


@pytest.mark.parametrize("name", list(CASES))
def test_tree_and_lists_bit_exact(name):
    x, y, o, g = pair_for(name)
    print("case", name, flush=True)
    assert np.array_equal(o.export(O.EX_SIZES), g.export("sizes"))
    assert np.array_equal(o.export(O.EX_LEVELS), g.export("levels"))
    assert np.array_equal(o.export(O.EX_PERM_X), g.export("perm_x"))
    assert np.array_equal(o.export(O.EX_PERM_Y), g.export("perm_y"))
    assert np.array_equal(o.nodes(), g.export("nodes").reshape(-1, 8))
    assert np.array_equal(o.boxes(), g.export("boxes").reshape(-1, 6))
    assert np.array_equal(o.L(), g.export("L").reshape(-1, 2))
    assert np.array_equal(o.Lm(), g.export("Lm").reshape(-1, 2))
    if CASES[name][1]["adm"] == "weak":
        assert np.array_equal(o.export(O.EX_NEAR_PTR), g.export("near_ptr"))
        assert np.array_equal(o.export(O.EX_NEAR_IDX), g.export("near_idx"))


def _deep_cluster(n, d, m, width, seed):
    """n uniform points plus m points inside a box of the given width: the
    tree descends about log2(1/width) stages around the cluster."""
    rng = np.random.default_rng(seed)
    x = rng.random((n + m, d))
    x[n:] = 0.3 + width * rng.random((m, d))
    return x


@pytest.mark.parametrize("case", ["2d_h2", "1d_hss", "1d_h2_xy"])
def test_tree_past_the_leading_key_bits(case):
    """The keys are first sorted by their leading 24 bits only (12 stages in
    2D, 24 in a binary tree); a tree that needs deeper stages is rebuilt from
    the full sort.  These point sets need 20-30 stages around a tight
    cluster, so they take that path: tree, permutation and lists must still
    equal the oracle's bit for bit, and the product its result."""
    if case == "2d_h2":
        x, y = _deep_cluster(3000, 2, 200, 1e-7, 21), None
        kw = dict(kernel="log_r", leaf=16, order=6, adm="strong", tol=1e-8, tau=0.7,
                  root=((0.0, 0.0), 1.0))
    elif case == "1d_hss":
        x, y = _deep_cluster(600, 1, 100, 1e-9, 22), None
        kw = dict(kernel="inv_r", leaf=8, order=8, adm="weak", tol=1e-9, eps_svd=1e-9,
                  tau=0.6, root=((0.0,), 1.0))
    else:
        x = _deep_cluster(800, 1, 120, 1e-9, 23)
        y = np.sort(_deep_cluster(700, 1, 90, 1e-9, 24), axis=0)
        kw = dict(kernel="exp_r", leaf=10, order=8, adm="strong", tol=1e-10, tau=0.6)
    o = O.Oracle(x, y, **_oracle_kwargs(kw))
    g = api.Smash(dev(x), None if y is None else dev(y), **kw)
    assert int(o.sizes()["nlevels"]) > (13 if x.shape[1] == 2 else 25)
    assert np.array_equal(o.export(O.EX_LEVELS), g.export("levels"))
    assert np.array_equal(o.export(O.EX_PERM_X), g.export("perm_x"))
    assert np.array_equal(o.export(O.EX_PERM_Y), g.export("perm_y"))
    assert np.array_equal(o.nodes(), g.export("nodes").reshape(-1, 8))
    assert np.array_equal(o.L(), g.export("L").reshape(-1, 2))
    assert np.array_equal(o.Lm(), g.export("Lm").reshape(-1, 2))
    q = W.rhs(g.ny, 3, seed=9)
    assert relerr(g.matvec(dev(q)).cpu().numpy(), o.matvec(q)) < 1e-10


def _split(arr, sizes):
    out, o = [], 0
    for s in sizes:
        out.append(arr[o:o + s])
        o += s
    return out


# HSS: the near-field vectors in C = [U-hat, S] are fixed only to about
# eps_mach / eps_svd by any SVD (eps_svd = 1e-9 .. 1e-10 here).  Against a
# 40-digit SVD of near blocks of these shapes, the oracle's Jacobi on the raw
# block misses the kept span by 1e-8 .. 5e-7 and the library's QR-first
# Jacobi by about a fifth of that; the pivot choices late in compr compare
# residual norms down to tol * |R11|, where that difference moves the
# relative gap between the two largest norms by up to ~1e-4.  A decision of
# compr or of the SVD truncation whose oracle margin is below HSS_TIE is
# therefore a genuine near-tie: the two skeleton choices are equally valid.
# The deciding quantity is named (pivot arg-max, rank cutoff against
# tol*|R11|, swap arg-max or rho against f, singular value against
# eps_svd*sigma_1), and the number of such nodes is bounded per case.
HSS_TIE = 1e-4
HSS_TIE_MAX_NODES = 3


def _gpu_per_node(g, side, nn):
    rk = g.export("ranks").reshape(-1, 6)
    mc, kc = (0, 1) if side == "row" else (2, 3)
    grid, sel, G = g.export(side + "_grid"), g.export(side + "_sel"), g.export(side + "_G")
    out = [(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, 0)))]
    og = og2 = 0
    for i in range(1, nn):
        m, k = int(rk[i, mc]), int(rk[i, kc])
        out.append((grid[og:og + m], sel[og:og + m], G[og2:og2 + (m - k) * k].reshape(m - k, k)))
        og += m
        og2 += (m - k) * k
    return out


def _hss_tie_subtrees(o, g, side, c):
    """Nodes whose results may differ from the oracle's: every node whose
    own result differs while one of its decisions is a near-tie in the
    oracle (margin < HSS_TIE; the decision is named), and its ancestors
    (their grids are built from it).  Any other difference fails, and so do
    more than HSS_TIE_MAX_NODES near-tie nodes per side."""
    ro, rg = o.ranks(), g.export("ranks").reshape(-1, 6)
    nodes = g.export("nodes").reshape(-1, 8)
    nn = nodes.shape[0]
    dm = o.export(O.EX_DECISION_MARGINS).reshape(-1, 8)[:, (0 if side == "row" else 4):][:, :4]
    po, pg = O.Oracle.per_node(o, side), _gpu_per_node(g, side, nn)
    tainted = np.zeros(nn, bool)
    ties = []
    for i in range(nn - 1, 0, -1):  # children come after their parents
        fc, nc_ = nodes[i, 2], nodes[i, 3]
        below = nc_ > 0 and tainted[fc:fc + nc_].any()
        same = (ro[i, c] == rg[i, c] and ro[i, c + 1] == rg[i, c + 1]
                and ro[i, 4 + c // 2] == rg[i, 4 + c // 2]
                and np.array_equal(po[i][0], pg[i][0]) and np.array_equal(po[i][1], pg[i][1]))
        if below:
            tainted[i] = True
        elif not same:
            d = int(np.argmin(dm[i]))
            assert dm[i, d] < HSS_TIE, (side, "node", i, "differs; oracle margins",
                                        dict(zip(O.DECISIONS, dm[i].tolist())))
            ties.append((i, O.DECISIONS[d], float(dm[i, d])))
            tainted[i] = True
    print("HSS near-tie nodes (%s side): %d %s; exempted with ancestors: %d of %d"
          % (side, len(ties), ties, int(tainted.sum()), nn - 1), flush=True)
    assert len(ties) <= HSS_TIE_MAX_NODES, ties
    return tainted


@pytest.mark.parametrize("name", list(CASES))
def test_ranks_skeletons_and_G(name):
    x, y, o, g = pair_for(name)
    print("case", name, flush=True)
    ro, rg = o.ranks(), g.export("ranks").reshape(-1, 6)
    sides = [("row", 0, O.EX_ROW_SEL, O.EX_ROW_G, O.EX_ROW_GRID)]
    if not (y is None and CASES[name][1]["kernel"] not in ("cauchy", "double_layer")):
        sides.append(("col", 2, O.EX_COL_SEL, O.EX_COL_G, O.EX_COL_GRID))
    weak = CASES[name][1]["adm"] == "weak"
    for side, c, exs, exg, exgrid in sides:
        m_o, k_o = ro[1:, c], ro[1:, c + 1]
        m_g, k_g = rg[1:, c], rg[1:, c + 1]
        if weak:
            keep = ~_hss_tie_subtrees(o, g, side, c)[1:]
        else:
            keep = np.ones(len(m_o), bool)
        # grids and ranks follow from the skeleton choices below them
        bad = np.nonzero(keep & ((m_o != m_g) | (k_o != k_g)))[0]
        assert bad.size == 0, (side, "first differing node", 1 + bad[:5])
        if weak:
            assert np.array_equal(ro[1:, 4 + c // 2][keep], rg[1:, 4 + c // 2][keep]), "SVD ranks"
        if keep.all():
            sel_o, sel_g = o.export(exs), g.export(side + "_sel")
            assert np.array_equal(o.export(exgrid), g.export(side + "_grid"))
            assert np.array_equal(sel_o, sel_g), side
        Go = _split(o.export(exg), (m_o - k_o) * k_o)
        Gg = _split(g.export(side + "_G"), (m_g - k_g) * k_g)
        if not weak:
            _check_h2_G(x, y, g, side, m_g, k_g, Go, Gg, CASES[name][1]["order"],
                        CASES[name][1].get("basis", "chebyshev"))
        else:
            _check_hss_ids(x, y, g, side, m_g, k_g, g.export(side + "_sel"), Go, Gg,
                           CASES[name][1]["order"], keep,
                           CASES[name][1].get("point_data") if side == "col" else None,
                           CASES[name][1].get("basis", "chebyshev"))


# H^2 G = (R11^-1 R12)^T against the oracle's, per node relative to
# max(1, |G|): 1e-10, the FP64 rule.  G solves a triangular system with R11,
# whose condition number equals that of the skeleton rows C_S of the basis
# and may reach about 1/tol; rounding then perturbs G by up to a small
# multiple of eps * cond(C_S) (the forward error of a backward-stable
# solve).  A node above 1e-10 must stay within 64 * eps * cond(C_S), with
# cond(C_S) computed here from the basis at the node's skeleton points.
H2_G_TOL = 1e-10


def _basis(pts, lo, hi, order, basis):
    """The far-field basis the construction used: interpolation (2.2) or, on
    the line, the Taylor basis (2.4)-(2.5)."""
    if basis == "taylor":
        return O.taylor_basis(pts, float(lo[0]), float(hi[0]), order)
    return O.interp_basis(pts, lo, hi, order)


def _check_h2_G(x, y, g, side, m, k, Go, Gg, order, basis="chebyshev"):
    P = x if side == "row" else (x if y is None else y)
    perm = g.export("perm_x" if side == "row" else "perm_y")
    grid = _split(g.export(side + "_grid"), m)
    sels = _split(g.export(side + "_sel"), m)
    bx = g.export("boxes").reshape(-1, 6)
    d = P.shape[1]
    worst, wide = 0.0, []
    for i, (a, b) in enumerate(zip(Go, Gg)):
        if not a.size:
            continue
        diff = float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(a))))
        worst = max(worst, diff)
        if diff < H2_G_TOL:
            continue
        node = i + 1
        U = _basis(P[perm[grid[i]]], bx[node, :d], bx[node, 3:3 + d], order, basis)
        cond = float(np.linalg.cond(U[sels[i][:int(k[i])]]))
        wide.append((node, diff, cond))
        assert diff <= 64 * np.finfo(np.float64).eps * cond, (side, node, diff, cond)
    print("H2 G worst difference", side, "%.2e" % worst,
          "; nodes above 1e-10 (node, diff, cond(C_S)):", wide, flush=True)


def _check_hss_ids(x, y, g, side, m, k, sel, Go, Gg, order, keep, pdata=None,
                   basis="chebyshev"):
    """HSS: C = [U-hat, S] contains near-field singular vectors whose trailing
    members (sigma near eps_svd * sigma_1) are fixed only to about
    eps_mach / eps_svd, so two correct implementations agree on the skeleton
    sets (checked above) but not on G to 1e-9.  Checked instead: the
    Gu-Eisenstat bound |G| <= f, and that G reproduces the far-field basis
    U-hat on the node's grid as well as the oracle's G does (ID residual,
    eq. (2.11)) -- at nodes inside a near-tie subtree (keep False) against
    the exact basis alone.  The product itself is held to 1e-10 elsewhere."""
    P = x if side == "row" else (x if y is None else y)
    perm = g.export("perm_x" if side == "row" else "perm_y")
    grid = _split(g.export(side + "_grid"), m)
    sels = _split(sel, m)
    bx = g.export("boxes").reshape(-1, 6)
    for i in range(len(m)):
        kk, mm = int(k[i]), int(m[i])
        if kk == 0 or kk == mm:
            continue
        node = i + 1
        assert np.max(np.abs(Gg[i])) <= 2.0 * (1 + 1e-8)
        pts = P[perm[grid[i]]]
        dd = P.shape[1]
        U = _basis(pts, bx[node, :dd], bx[node, 3:3 + dd], order, basis)
        if pdata is not None:  # double-layer column side: [m_1 U-hat, m_2 U-hat]
            md = pdata[perm[grid[i]]]
            U = np.concatenate([U * md[:, :1], U * md[:, 1:2]], axis=1)
        sk, rs = sels[i][:kk], sels[i][kk:]
        Gg_ = Gg[i].reshape(mm - kk, kk)
        nrm = np.linalg.norm(U)
        r_g = np.linalg.norm(U[rs] - Gg_ @ U[sk])
        if keep[i]:
            Go_ = Go[i].reshape(mm - kk, kk)
            r_o = np.linalg.norm(U[rs] - Go_ @ U[sk])
            assert r_g <= 10.0 * r_o + 1e-12 * nrm, (node, r_g, r_o)
        else:
            assert r_g <= 1e-6 * nrm, (node, r_g)


@pytest.mark.parametrize("name", list(CASES))
def test_coupling_blocks_are_kernel_entries(name):
    """B_ij = A(X at i-hat, Y at j-hat) over L, stored column-major."""
    x, y, o, g = pair_for(name)
    yy = x if y is None else y
    kw = CASES[name][1]
    L = g.export("L").reshape(-1, 2)
    B = g.export("coupling")
    rk = g.export("ranks").reshape(-1, 6)
    px, py = g.export("perm_x"), g.export("perm_y")
    # at the library's own skeletons (they equal the oracle's, up to the
    # near-ties allowed above)
    reuse = y is None and kw["kernel"] not in ("cauchy", "double_layer")
    pdata = kw.get("point_data")
    per_r = _gpu_per_node(g, "row", rk.shape[0])
    per_c = per_r if reuse else _gpu_per_node(g, "col", rk.shape[0])
    off = 0
    rng = np.random.default_rng(0)
    pick = set(rng.choice(len(L), size=min(len(L), 200), replace=False).tolist())
    for e, (i, j) in enumerate(L):
        ki, kj = rk[i, 1], rk[j, 3]
        if e in pick:
            gi, si, _ = per_r[i]
            gj, sj, _ = per_c[j]
            ir, jc = px[gi[si[:ki]]], py[gj[sj[:kj]]]
            rows, cols = x[ir], yy[jc]
            ref = O.kernel_block(rows, cols, kw["kernel"],
                                 data_P=None if pdata is None else pdata[ir],
                                 data_Q=None if pdata is None else pdata[jc])
            blk = B[off:off + ki * kj].reshape(kj, ki).T
            assert np.max(np.abs(blk - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
        off += ki * kj
    assert off == B.size


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("nrhs", [1, 3, 16, 70])
def test_matvec_fp64_parity(name, nrhs):
    x, y, o, g = pair_for(name)
    print("case", name, nrhs, flush=True)
    q = W.rhs(g.ny, nrhs, seed=nrhs)
    z_o = o.matvec(q)
    z_g = g.matvec(dev(q)).cpu().numpy()
    assert relerr(z_g, z_o) < 1e-10


def test_matvec_strided_input_and_vector():
    x, y, o, g = pair_for("h2_2d_log")
    q = W.rhs(g.ny, 24, seed=7)
    Q = dev(q)
    z = g.matvec(Q[:, 4:20])  # leading dimension 24 > nrhs
    assert relerr(z.cpu().numpy(), o.matvec(q[:, 4:20])) < 1e-10
    zv = g.matvec(Q[:, 5].contiguous())
    assert relerr(zv.cpu().numpy(), o.matvec(q[:, 5])) < 1e-10


@pytest.mark.parametrize("name", ["h2_2d_log", "hss1d_small", "h2_3d_clusters"])
def test_plain_per_node_form_equals_batched(name):
    x, y, o, g = pair_for(name)
    kw = dict(CASES[name][1])
    gp = api.Smash(dev(x), None if y is None else dev(y), batched=False, **kw)
    for what in ("perm_x", "nodes", "L", "Lm", "ranks", "row_sel"):
        assert np.array_equal(gp.export(what), g.export(what))
    assert np.array_equal(gp.export("row_G"), g.export("row_G"))
    q = dev(W.rhs(g.ny, 5, seed=2))
    assert torch.equal(gp.matvec(q), g.matvec(q))


@pytest.mark.parametrize("name", ["h2_2d_log", "h2_3d_clusters", "hss_cauchy_xy"])
@pytest.mark.parametrize("eval_prec", ["f64", "f32"])
def test_matvec_fp32_apply(name, eval_prec):
    """FP32 apply, with the blocks evaluated in FP64 (then rounded) or by the
    FP32 kernel arithmetic on FP64 coordinate differences (the form the
    large workloads run): within 1e-5 relative Frobenius of the FP64
    oracle's product on the FP32-rounded right-hand sides."""
    mk, kw = CASES[name]
    x, y = mk()
    o = O.Oracle(x, y, **_oracle_kwargs(kw))
    g = api.Smash(dev(x), None if y is None else dev(y), apply_prec="f32", eval_prec=eval_prec,
                  **kw)
    print("case", name, eval_prec, flush=True)
    for nrhs in (1, 16, 64):
        q32 = W.rhs(g.ny, nrhs, seed=3).astype(np.float32)
        z_o = o.matvec(q32.astype(np.float64))
        z_g = g.matvec(torch.from_numpy(q32).cuda()).cpu().numpy().astype(np.float64)
        e = relerr(z_g, z_o)
        print("  nrhs", nrhs, "rel. error vs FP64 oracle %.2e" % e, flush=True)
        assert e < 1e-5, nrhs
    g.close()


@pytest.mark.parametrize("name", [c for c in CASES if c not in DL])
def test_evaluated_coupling_fp64_parity(name):
    """The index-only form (coupling blocks re-evaluated from the skeleton
    points inside each product, a chunk of pairs at a time) against the FP64
    oracle, whose product evaluates every block on the fly: within 1e-10."""
    x, y, o, _ = pair_for(name)
    kw = CASES[name][1]
    g = api.Smash(dev(x), None if y is None else dev(y), coupling="evaluated",
                  coupling_chunk=5000, **kw)
    print("case", name, flush=True)
    for nrhs in (1, 16):
        q = W.rhs(g.ny, nrhs, seed=30 + nrhs)
        z_o = o.matvec(q)
        for _ in range(2):  # eager, then captured
            z_g = g.matvec(dev(q)).cpu().numpy()
            assert relerr(z_g, z_o) < 1e-10, nrhs
    g.close()


@pytest.mark.parametrize("name", ["h2_2d_log", "h2_3d_clusters", "hss_cauchy_xy", "hss1d_cfg"])
def test_matvec_bf16_apply(name):
    """BF16 G copies and blocks on the BF16 matrix cores with FP32 vectors and
    accumulation.  BF16 keeps 8 significand bits (unit roundoff 2^-9), so the
    product is expected within a few 1e-3 of the FP64 oracle; the bound is
    2e-2.  The construction is the FP64 one: skeletons equal the oracle's."""
    mk, kw = CASES[name]
    x, y = mk()
    o = O.Oracle(x, y, **_oracle_kwargs(kw))
    g = api.Smash(dev(x), None if y is None else dev(y), apply_prec="bf16", eval_prec="f32",
                  **kw)
    assert np.array_equal(g.export("ranks").reshape(-1, 6)[1:, :4], o.ranks()[1:, :4])
    errs = []
    for nrhs in (1, 16, 40, 64):
        q32 = W.rhs(g.ny, nrhs, seed=4).astype(np.float32)
        z_o = o.matvec(q32.astype(np.float64))
        z_g = g.matvec(torch.from_numpy(q32).cuda()).cpu().numpy().astype(np.float64)
        assert np.isfinite(z_g).all()
        errs.append(relerr(z_g, z_o))
    print(name, "BF16 apply rel. error vs FP64 oracle", ["%.2e" % e for e in errs])
    assert max(errs) < 2e-2, errs


@pytest.mark.parametrize("name", ["h2_2d_log", "hss1d_cfg", "hss_cauchy_xy", "h2_3d_clusters"])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_evaluated_coupling_equals_stored(name, prec):
    """Coupling blocks evaluated inside each product -- by each lane right
    before its matrix-core step (FP64, FP32 apply), or a chunk of pairs at a
    time through a workspace (BF16 apply; chunks of 3000 entries here, so
    every product runs many chunks and chunks end inside a row node's pair
    range) -- give the product of the stored blocks bit for bit: the same
    block values enter the same contraction.  Also checks the bookkeeping
    through smash_info and that the exported (re-evaluated) blocks equal the
    stored ones."""
    mk, kw = CASES[name]
    x, y = mk()
    ev = "f64" if prec == "f64" else "f32"
    X, Y = dev(x), None if y is None else dev(y)
    gs = api.Smash(X, Y, apply_prec=prec, eval_prec=ev, coupling="stored", **kw)
    ge = api.Smash(X, Y, apply_prec=prec, eval_prec=ev, coupling="evaluated",
                   coupling_chunk=3000, **kw)
    ie, is_ = ge.info(), gs.info()
    assert is_["coupling_evaluated"] == 0
    if is_["coupling_entries"] > 0:
        assert ie["coupling_evaluated"] == 1
        if prec == "bf16":  # a chunk of pairs at a time through a workspace
            assert ie["coupling_chunks"] >= is_["coupling_entries"] // 3000
            assert 3000 <= ie["coupling_ws_entries"] or ie["coupling_chunks"] == 1
            if ie["coupling_chunks"] > 2:
                assert ie["coupling_ws_entries"] < is_["coupling_entries"]
        else:  # evaluated inside the contraction: no workspace
            assert ie["coupling_chunks"] == 0 and ie["coupling_ws_entries"] == 0
            assert ie["device_bytes"] < is_["device_bytes"]
    dt = torch.float64 if prec == "f64" else torch.float32
    for nrhs in (1, 16, 40):
        q = torch.from_numpy(W.rhs(gs.ny, nrhs, seed=6)).to(dt).cuda()
        zs = gs.matvec(q).cpu().numpy()
        for _ in range(3):  # eager, then captured and replayed
            ze = ge.matvec(q).cpu().numpy()
            assert np.array_equal(zs, ze), (name, prec, nrhs)
    if prec != "bf16":
        assert np.array_equal(gs.export("coupling"), ge.export("coupling"))


def test_full_size_h2_2d_log_65536():
    """The benchmark workload at full size: bit-exact tree/lists/skeletons,
    FP64 product within 1e-10 of the oracle, and within the tolerance of
    exact rows of A Q."""
    cfg = W.CONFIGS["h2_2d_log_65536"]
    x, _ = W.points(cfg)
    kw = dict(kernel="log_r", leaf=64, order=8, adm="strong", tol=1e-8, tau=0.7,
              root=((0.0, 0.0), 1.0))
    o = O.Oracle(x, **_oracle_kwargs(kw))
    g = api.Smash(dev(x), **kw)
    for what, ex in (("perm_x", O.EX_PERM_X), ("levels", O.EX_LEVELS), ("L", O.EX_L),
                     ("Lm", O.EX_LM), ("row_sel", O.EX_ROW_SEL)):
        assert np.array_equal(o.export(ex), g.export(what)), what
    q = W.rhs(cfg["n"], cfg["nrhs"])
    z_o = o.matvec(q)
    z_g = g.matvec(dev(q)).cpu().numpy()
    assert relerr(z_g, z_o) < 1e-10
    rows = np.arange(0, cfg["n"], 257)
    zr = O.dense_rows(x, x, rows, q, "log_r")
    assert relerr(z_g[rows], zr) < 1e-6


def _full_size(name, nrhs, rows_every, bound, apply_prec="f32"):
    cfg = W.CONFIGS[name]
    x, y = W.points(cfg)
    kw = dict(kernel=cfg["kernel"], leaf=cfg["leaf"], order=cfg["order"],
              adm="strong" if cfg["adm"] == 1 else "weak", tol=cfg["tol"], tau=cfg["tau"],
              root=cfg["root"], apply_prec=apply_prec,
              eval_prec="f64" if apply_prec == "f64" else "f32")
    if "eps_svd" in cfg:
        kw["eps_svd"] = cfg["eps_svd"]
    print("case", name, apply_prec, flush=True)
    g = api.Smash(dev(x), None if y is None else dev(y), **kw)
    px = g.export("perm_x")
    assert np.array_equal(np.sort(px), np.arange(cfg["n"]))
    yy = x if y is None else y
    q = W.rhs(len(yy), nrhs).astype(np.float32)
    z = g.matvec(torch.from_numpy(q).cuda()).cpu().numpy().astype(np.float64)
    g.close()
    rows = np.arange(0, cfg["n"], rows_every)
    zr = O.dense_rows(x, yy, rows, q.astype(np.float64), cfg["kernel"])
    err = relerr(z[rows], zr)
    print(name, apply_prec, "rel. error vs exact rows", err, flush=True)
    assert err < bound, err


def test_full_size_h2_3d_clusters_1m():
    """The 3D clustered workload at full size (2^20 points, 64 FP32 right-hand
    sides; the handle holds about 156 GB): every product row sampled is
    within 2e-5 of the exact row (tol 1e-6; measured 4.7e-6), and BF16 apply
    within 2e-2."""
    _full_size("h2_3d_inv_r_clusters_1m", 64, 4096, 2e-5)
    _full_size("h2_3d_inv_r_clusters_1m", 64, 4096, 2e-2, "bf16")


def test_full_size_hss_cauchy_1m():
    """The Cauchy HSS workload at full size (2^20 points, X != Y): sampled
    product rows within 1e-6 of the exact rows (measured 1.4e-7)."""
    _full_size("hss1d_cauchy_1m", 16, 4096, 1e-6)


def test_single_leaf_and_tiny_inputs():
    for n in (1, 2, 7, 64):
        x = W.uniform(n, 2, n)
        g = api.Smash(dev(x), kernel="inv_r", leaf=64, order=4, adm="strong", tol=1e-6,
                      root=((0.0, 0.0), 1.0))
        q = W.rhs(n, 2)
        zd = O.dense_matvec(x, x, q, "inv_r")
        assert relerr(g.matvec(dev(q)).cpu().numpy(), zd) < 1e-14


def test_errors_from_device_checks():
    x = W.uniform(100, 2, 0) * 2.0
    with pytest.raises(api.SmashError) as e:
        api.Smash(dev(x), kernel="inv_r", leaf=8, order=4, adm="strong", tol=1e-6,
                  root=((0.0, 0.0), 1.0))
    assert e.value.code == -1
    x = W.uniform(100, 2, 0)
    x[5, 1] = np.nan
    with pytest.raises(api.SmashError) as e:
        api.Smash(dev(x), kernel="inv_r", leaf=8, order=4, adm="strong", tol=1e-6)
    assert e.value.code == -5


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_matvec_graph_replays_match_eager(prec):
    """The product replayed from its captured HIP graph equals the eager
    launch sequence bit for bit, on every replay, with eager work and
    synchronizations in between; a new argument set or a larger workspace
    captures again."""
    mk, kw = CASES["h2_2d_log"]
    x, _ = mk()
    dt = torch.float64 if prec == "f64" else torch.float32
    ev = "f64" if prec == "f64" else "f32"
    ge = api.Smash(dev(x), apply_prec=prec, eval_prec=ev, graphs=False, **kw)
    gg = api.Smash(dev(x), apply_prec=prec, eval_prec=ev, graphs=True, **kw)
    for nrhs in (16, 80):
        Q = dev(W.rhs(len(x), nrhs, seed=11)).to(dt)
        Q2 = dev(W.rhs(len(x), nrhs, seed=12)).to(dt)
        ref = ge.matvec(Q)
        out = torch.empty_like(ref)
        for rep in range(5):
            gg.matvec(Q, out=out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (nrhs, rep)
            other = ge.matvec(Q2)  # eager work between replays
            torch.cuda.synchronize()
            assert torch.isfinite(other).all()
    inf = gg.info()
    assert inf["graph_captures"] == 2 and inf["graph_replays"] == 8, inf
    gg.close()
    ge.close()


def test_autotuner_shape_keeps_the_product():
    """The tuner returns one of its candidate shapes, and the product with
    the tuned shape equals the default-shape product up to the summation
    order of the split sweeps."""
    from paper_1705_05443_amd import autotune
    mk, kw = CASES["h2_2d_log"]
    x, _ = mk()
    res = autotune.tune(x, None, nrhs=16, reps=2, **kw)
    shp = res["shape"]
    assert shp["mv_split_nodes"] in autotune.KNOBS["mv_split_nodes"]
    assert shp["mv_xcd_run"] in autotune.KNOBS["mv_xcd_run"]
    assert len(res["trials"]) == sum(len(v) for v in autotune.KNOBS.values())
    q = dev(W.rhs(len(x), 16, seed=21))
    g0 = api.Smash(dev(x), tuned=False, **kw)
    g1 = api.Smash(dev(x), tuned=False, **kw, **shp)
    z0, z1 = g0.matvec(q).cpu().numpy(), g1.matvec(q).cpu().numpy()
    assert relerr(z1, z0) < 1e-13


@pytest.mark.parametrize("scale", [1e-155, 1e140])
def test_log_kernel_blocks_at_extreme_scales(scale):
    """log|x - y| blocks where |x - y|^2 is subnormal (points in a box of side
    1e-155) or near the top of the range (side 1e140), against numpy's log
    of the same FP64 squared distance: the library's logarithm (argument
    reduction and the atanh series) stays within a few units in the last
    place there too."""
    x = W.uniform(3000, 2, 21) * scale
    g = api.Smash(dev(x), kernel="log_r", leaf=64, order=6, adm="strong", tol=1e-6, tau=0.7,
                  root=((0.0, 0.0), scale), graphs=False)
    print("scale", scale, flush=True)
    L = g.export("L").reshape(-1, 2)
    B = g.export("coupling")
    rk = g.export("ranks").reshape(-1, 6)
    px = g.export("perm_x")
    per = _gpu_per_node(g, "row", rk.shape[0])
    assert len(L) > 0
    off, worst = 0, 0.0
    for i, j in L:
        ki, kj = rk[i, 1], rk[j, 1]
        gi, si, _ = per[i]
        gj, sj, _ = per[j]
        rows = x[px[gi[si[:ki]]]]
        cols = x[px[gj[sj[:kj]]]]
        d = rows[:, None, :] - cols[None, :, :]
        ref = 0.5 * np.log(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1])
        blk = B[off:off + ki * kj].reshape(kj, ki).T
        worst = max(worst, float(np.max(np.abs(blk - ref) / np.abs(ref))))
        off += ki * kj
    g.close()
    assert off == B.size
    assert worst < 8 * np.finfo(np.float64).eps, worst


def test_batched_products_equal_single_ones():
    """smash_matvec_batched over several handles (one of them twice, the
    second time with another right-hand side) gives each product bit for bit
    as smash_matvec does."""
    import torch
    specs = [(W.uniform(4000, 2, 31), dict(kernel="log_r", leaf=64, order=8, adm="strong",
                                            tol=1e-8, tau=0.7, root=((0.0, 0.0), 1.0))),
             (W.uniform(3000, 1, 32), dict(kernel="inv_r", leaf=32, order=10, adm="weak",
                                            tol=1e-9, tau=0.6, root=((0.0,), 1.0)))]
    hs = [api.Smash(dev(x), **kw) for x, kw in specs]
    rng = np.random.default_rng(5)
    order = [0, 1, 0]
    Xs = [torch.from_numpy(rng.standard_normal((hs[c].ny, r))).cuda()
          for c, r in zip(order, (3, 16, 7))]
    print("batched products of", [hs[c].ny for c in order], flush=True)
    single = [hs[c].matvec(X).cpu().numpy() for c, X in zip(order, Xs)]
    outs = [torch.empty((hs[c].nx, X.shape[1]), dtype=torch.float64, device="cuda")
            for c, X in zip(order, Xs)]
    for rep in range(3):  # eager, captured, replayed (same argument sets)
        batched = api.matvec_batched([hs[c] for c in order], Xs, outs)
        torch.cuda.synchronize()
        for a, b in zip(single, batched):
            assert np.array_equal(a, b.cpu().numpy())
    for h in hs:
        h.close()


def test_allocator_hooks_take_every_device_allocation():
    """With torch's caching allocator as the hooks, a handle's memory shows in
    torch's accounting while it lives, every allocation is given back at
    destroy, the build's peak in smash_info equals the most the hooks held
    during the construction, and the product equals the one of a handle on
    the library's own pool bit for bit (also after smash_trim)."""
    import ctypes as C
    import torch
    x = W.uniform(5000, 2, 41)
    kw = dict(kernel="log_r", leaf=64, order=8, adm="strong", tol=1e-8, tau=0.7,
              root=((0.0, 0.0), 1.0))
    live = {}
    most = [0]
    talloc, tfree = api.torch_allocator_hooks()

    def _alloc(ctx, n, s):
        p = talloc(ctx, n, s)
        if p:
            live[p] = n
            most[0] = max(most[0], sum(live.values()))
        return p

    def _free(ctx, p, n, s):
        assert live.pop(p) == n
        tfree(ctx, p, n, s)

    hooks = (api.ALLOC_FN(_alloc), api.FREE_FN(_free))
    q = torch.from_numpy(np.random.default_rng(2).standard_normal((5000, 4))).cuda()
    print("hooks build", flush=True)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    h = api.Smash(dev(x), allocator=hooks, **kw)
    held = sum(live.values())
    inf = h.info()
    assert held >= inf["device_bytes"] > 0
    assert inf["build_peak_bytes"] == most[0] >= held, (inf["build_peak_bytes"], most[0], held)
    z = h.matvec(q).cpu().numpy()
    assert torch.cuda.memory_allocated() - before >= held
    h.close()
    assert not live  # every allocation went back through the hook
    g = api.Smash(dev(x), **kw)
    assert np.array_equal(g.matvec(q).cpu().numpy(), z)
    assert g.info()["build_peak_bytes"] >= g.info()["device_bytes"]
    g.close()
    api.trim()
    g = api.Smash(dev(x), **kw)
    assert np.array_equal(g.matvec(q).cpu().numpy(), z)
    g.close()


def test_allocation_failure_reports_oom_and_frees_everything():
    """A device allocation that fails in the middle of a construction (the
    allocator hook returns NULL at its first, a middle and its last call)
    ends the build with SMASH_E_OOM, and every allocation granted before it
    is given back; a product whose workspace allocation fails reports the
    same and leaves the handle usable."""
    import torch
    x = W.clusters(6000, 3, 12)
    kw = dict(kernel="inv_r", leaf=128, order=5, adm="strong", tol=1e-6, tau=0.7,
              root=((0.0, 0.0, 0.0), 1.0))
    talloc, tfree = api.torch_allocator_hooks()
    state = {"calls": 0, "fail_at": -1, "live": {}}

    def _alloc(ctx, n, s):
        state["calls"] += 1
        if state["calls"] == state["fail_at"]:
            return None
        p = talloc(ctx, n, s)
        if p:
            state["live"][p] = n
        return p

    def _free(ctx, p, n, s):
        assert state["live"].pop(p) == n
        tfree(ctx, p, n, s)

    hooks = (api.ALLOC_FN(_alloc), api.FREE_FN(_free))
    X = dev(x)
    h = api.Smash(X, allocator=hooks, **kw)  # count the calls of a whole build
    total = state["calls"]
    q = torch.from_numpy(np.random.default_rng(3).standard_normal((6000, 8))).cuda()
    z_ok = h.matvec(q).cpu().numpy()
    h.close()
    assert not state["live"] and total > 2
    for fail_at in (1, total // 2, total):
        state.update(calls=0, fail_at=fail_at)
        print("build, allocation %d of %d fails" % (fail_at, total), flush=True)
        with pytest.raises(api.SmashError) as e:
            api.Smash(X, allocator=hooks, **kw)
        assert e.value.code == -3, str(e.value)  # SMASH_E_OOM
        torch.cuda.synchronize()
        assert not state["live"], len(state["live"])
    # a product whose workspace allocation fails
    state.update(calls=0, fail_at=-1)
    h = api.Smash(X, allocator=hooks, **kw)
    state.update(calls=0, fail_at=1)
    with pytest.raises(api.SmashError) as e:
        h.matvec(torch.from_numpy(np.random.default_rng(4).standard_normal((6000, 40))).cuda())
    assert e.value.code == -3, str(e.value)
    state.update(fail_at=-1)
    assert np.array_equal(h.matvec(q).cpu().numpy(), z_ok)
    h.close()
    torch.cuda.synchronize()
    assert not state["live"]


def test_levels_wider_than_one_workgroup():
    """Tree levels of more than 4096 nodes take the multi-workgroup form of
    the level bookkeeping (sizes, capacities, slot offsets) instead of the
    one-workgroup form; both must give the oracle's ranks and product."""
    x = W.uniform(80000, 2, 51)
    kw = dict(kernel="log_r", leaf=8, order=4, adm="strong", tol=1e-6, tau=0.7,
              root=((0.0, 0.0), 1.0))
    o = O.Oracle(x, None, **_oracle_kwargs(kw))
    lv = o.export(O.EX_LEVELS)
    assert np.max(np.diff(lv)) > 4096 >= np.min(np.diff(lv))  # both forms run
    print("level sizes", np.diff(lv).tolist(), flush=True)
    g = api.Smash(dev(x), **kw)
    assert np.array_equal(o.export(O.EX_LEVELS), g.export("levels"))
    ro, rg = o.ranks(), g.export("ranks").reshape(-1, 6)
    assert np.array_equal(ro[:, :2], rg[:, :2])
    q = W.rhs(g.ny, 3, seed=4)
    z_o = o.matvec(q)
    z_g = g.matvec(dev(q)).cpu().numpy()
    g.close()
    assert relerr(z_g, z_o) < 1e-10


def test_products_of_one_handle_on_two_streams_are_ordered():
    """Products of one handle share its workspace.  Enqueued on two streams
    with no synchronisation between them -- the second one needing a larger
    workspace, which the library then grows -- each still equals the same
    product run alone, because the library orders a handle's products."""
    x, _ = CASES["h2_2d_log"][0]()
    kw = CASES["h2_2d_log"][1]
    ref_h = api.Smash(dev(x), graphs=False, **kw)
    h = api.Smash(dev(x), **kw)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    Qs = [dev(W.rhs(len(x), r, seed=40 + r)) for r in (16, 80, 5, 16)]
    refs = [ref_h.matvec(Q) for Q in Qs]
    torch.cuda.synchronize()
    for rep in range(3):
        outs = [torch.empty_like(r) for r in refs]
        for c, (Q, o) in enumerate(zip(Qs, outs)):
            h.matvec(Q, out=o, stream=s1 if c % 2 == 0 else s2)
        torch.cuda.synchronize()
        for c, (o, r) in enumerate(zip(outs, refs)):
            assert torch.equal(o, r), (rep, c)
    h.close()
    ref_h.close()


@pytest.mark.parametrize("name", ["h2_2d_log", "hss1d_cfg", "hss_cauchy_xy", "hss_dl_ram_head"])
def test_storage_accounting(name):
    """smash_info's storage comparison (Sec. 6.6, Table 6.6): recomputed here
    from the exported ranks and lists -- the dense matrix, the generators as
    dense matrices (HSS0), and G with the index sets (B fixed by the
    skeletons) -- and SMASH below HSS0 below the dense matrix."""
    x, y, o, g = pair_for(name)
    inf = g.info()
    rk = g.export("ranks").reshape(-1, 6)[1:]
    sides = [(0, 1)] if inf["symmetric_reuse"] else [(0, 1), (2, 3)]
    mk = sum(int(np.sum(rk[:, a].astype(np.int64) * rk[:, b])) for a, b in sides)
    gk = sum(int(np.sum((rk[:, a] - rk[:, b]).astype(np.int64) * rk[:, b])) for a, b in sides)
    sm = sum(int(np.sum(rk[:, a].astype(np.int64))) for a, _ in sides)
    nL, nLm = len(g.export("L")) // 2, len(g.export("Lm")) // 2
    assert inf["bytes_dense"] == 8 * inf["nx"] * inf["ny"]
    assert inf["bytes_hss0"] == 8 * (mk + inf["coupling_entries"] + inf["near_entries"])
    assert inf["bytes_smash"] == 8 * (gk + inf["near_entries"]) + 4 * (sm + 2 * (nL + nLm))
    print(name, "storage MB: dense %.1f HSS0 %.2f SMASH %.2f" % (
        inf["bytes_dense"] / 1e6, inf["bytes_hss0"] / 1e6, inf["bytes_smash"] / 1e6))
    assert inf["bytes_smash"] < inf["bytes_hss0"] < inf["bytes_dense"]


@pytest.mark.parametrize("scale", [1e-140, 1.0, 1e130])
def test_inv_r_kernel_blocks_against_numpy(scale):
    """1/|x - y| blocks (the library's reciprocal square root: the hardware
    estimate and two Newton-Raphson steps) against numpy's 1/sqrt of the same
    FP64 squared distance, at unit scale and where |x - y|^2 is near the
    ends of the range the refinement takes (below 2^-900 and above 2^900 it
    falls back to a square root and a division): within 2 units in the last
    place."""
    x = W.uniform(3000, 3, 23) * scale
    g = api.Smash(dev(x), kernel="inv_r", leaf=64, order=3, adm="strong", tol=1e-6, tau=0.7,
                  root=((0.0, 0.0, 0.0), scale), graphs=False)
    L = g.export("L").reshape(-1, 2)
    B = g.export("coupling")
    rk = g.export("ranks").reshape(-1, 6)
    px = g.export("perm_x")
    per = _gpu_per_node(g, "row", rk.shape[0])
    assert len(L) > 0
    off, worst = 0, 0.0
    for i, j in L:
        ki, kj = rk[i, 1], rk[j, 1]
        gi, si, _ = per[i]
        gj, sj, _ = per[j]
        rows = x[px[gi[si[:ki]]]]
        cols = x[px[gj[sj[:kj]]]]
        d = rows[:, None, :] - cols[None, :, :]
        ref = 1.0 / np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2])
        blk = B[off:off + ki * kj].reshape(kj, ki).T
        worst = max(worst, float(np.max(np.abs(blk - ref) / ref)))
        off += ki * kj
    g.close()
    assert off == B.size
    print("scale", scale, "worst relative difference %.2e" % worst, flush=True)
    assert worst < 2 * np.finfo(np.float64).eps, worst


def test_double_layer_gpu_against_dense_and_gauss():
    """The double-layer HSS matrix on the GPU (ram head, n = 2560): its
    product reproduces the dense Nystrom matrix within Table 6.3's
    ||A - A_hat||_max order, the rows of K - I/2 sum to -1 (Gauss's
    integral), and coupling requests for the evaluated form are refused."""
    pts, data = W.curve("ram_head", 2560)
    kw = dict(kernel="double_layer", leaf=50, order=5, adm="weak", tol=1e-10, eps_svd=1e-11,
              tau=0.6)
    g = api.Smash(dev(pts), point_data=dev(data), **kw)
    one = g.matvec(torch.ones(2560, 1, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert np.max(np.abs(one + 1.0)) < 1e-8
    A = O.kernel_block(pts, pts, "double_layer", data_P=data, data_Q=data)
    Ah = g.matvec(dev(np.eye(2560))).cpu().numpy()
    err = float(np.max(np.abs(A - Ah)))
    print("double layer ram head 2560: ||A - A_hat||_max %.2e" % err, flush=True)
    assert err < 1e-9
    g.close()
    with pytest.raises(api.SmashError) as e:
        api.Smash(dev(pts), point_data=dev(data), coupling="evaluated", **kw)
    assert e.value.code == -2


def test_taylor_basis_needs_points_on_the_line():
    """The Taylor basis of eqs. (2.4)-(2.5) is defined here for points on the
    line only: a 2D build asking for it is refused with SMASH_E_UNSUPPORTED."""
    x = W.uniform(500, 2, 1)
    with pytest.raises(api.SmashError) as e:
        api.Smash(dev(x), kernel="log_r", leaf=32, order=6, adm="strong", tol=1e-8,
                  basis="taylor")
    assert e.value.code == -2
    with pytest.raises(ValueError):
        api.Smash(dev(W.uniform(500, 1, 1)), basis="legendre")


def test_order_for_a_tolerance_is_the_smallest_that_reaches_it():
    """autotune.order_for: the returned order's product is within the tolerance
    of exact rows and every smaller order tried is not; its exact rows equal
    the oracle's dense rows (1/r in 3D, log r in 2D, 1/(x - y) on the line)."""
    from paper_1705_05443_amd import autotune
    x2 = W.uniform(6000, 2, 3)
    p, err, tried = autotune.order_for(x2, kernel="log_r", tol=1e-6, leaf=64, adm="strong",
                                       tau=0.7, root=((0.0, 0.0), 1.0))
    print("log r 2D orders tried", tried, flush=True)
    assert err <= 1e-6 and len(tried) >= 2
    assert all(e > 1e-6 for _, e in tried[:-1])
    x3 = W.clusters(6000, 3, 4)
    p3, err3, tried3 = autotune.order_for(x3, kernel="inv_r", tol=1e-6, leaf=128,
                                          adm="strong", tau=0.7, root=((0.0, 0.0, 0.0), 1.0),
                                          orders=range(3, 9))  # p^3 <= 512 basis columns
    print("1/r 3D orders tried", tried3, flush=True)
    assert err3 <= 1e-6 and all(e > 1e-6 for _, e in tried3[:-1])
    q = W.rhs(6000, 2, seed=5)
    rows = np.arange(0, 6000, 97)
    for xx, yy, kern in ((x3, None, "inv_r"), (x2, None, "log_r"),
                         (*W.chebyshev_pair(6000, 2), "cauchy")):
        zr = autotune.exact_rows(xx, yy, rows, q, kern)
        zo = O.dense_rows(xx, xx if yy is None else yy, rows, q, kern)
        assert relerr(zr, zo) < 1e-12, kern

