// pairs.hip -- admissible leaves L and inadmissible leaves L^- (eqs. (3.3),
// (3.4); HSS form eq. (3.5)) and the HSS near-field sets N_i (eq. (A.1)).
//
// H^2: level-synchronous dual traversal from (root, root).  Every frontier
// pair is classified in parallel -- distinct and well separated: L; two
// leaves: L^-; two inner nodes (then always on one level): all child pairs;
// a leaf and an inner node: the leaf against the inner node's children --
// and the next frontier is compacted with scans.  The lists are then sorted
// by (i, j) with the stable radix sort, so they are bit-exact regardless of
// emission order.
#include "common.cuh"

namespace smash {

struct TreeView {
  const int *level, *parent, *first_child, *nchild, *xb, *xe, *yb, *ye;
  const double *lo, *hi;
};

static TreeView view(const Handle &h) {
  return TreeView{h.level, h.parent, h.first_child, h.nchild, h.xb, h.xe, h.yb, h.ye, h.lo, h.hi};
}

__global__ void k_front_count(TreeView T, const int *fi, const int *fj, int64_t nf, int d,
                              double tau, int64_t *cL, int64_t *cLm, int64_t *cE) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int i = fi[f], j = fj[f];
  int l = 0, lm = 0;
  int64_t e = 0;
  int ni = T.nchild[i], nj = T.nchild[j];
  if (i != j && well_separated(T.lo, T.hi, i, j, d, tau))
    l = 1;
  else if (ni == 0 && nj == 0)
    lm = 1;
  else if (ni > 0 && nj > 0)
    e = (int64_t)ni * nj;
  else
    e = ni == 0 ? nj : ni;
  cL[f] = l;
  cLm[f] = lm;
  cE[f] = e;
}

// o: exclusive scan of the concatenated counts (L, L^-, expansion) of the
// nf frontier pairs; tL, tLm: the totals of the first and of the first two
// segments.  L and L^- pairs are written at their offsets in Li/Lj and
// Lmi/Lmj (the callers' running positions), expansions into ni/nj.
__global__ void k_front_emit(TreeView T, const int *fi, const int *fj, int64_t nf,
                             const int64_t *o, int64_t tL, int64_t tLm, int *Li, int *Lj,
                             int *Lmi, int *Lmj, int *ni_out, int *nj_out) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int i = fi[f], j = fj[f];
  if (o[f + 1] > o[f]) {
    Li[o[f]] = i;
    Lj[o[f]] = j;
    return;
  }
  if (o[nf + f + 1] > o[nf + f]) {
    Lmi[o[nf + f] - tL] = i;
    Lmj[o[nf + f] - tL] = j;
    return;
  }
  int64_t o_ = o[2 * nf + f] - tLm;
  int ni = T.nchild[i], nj = T.nchild[j];
  if (ni > 0 && nj > 0) {
    for (int c = 0; c < ni; c++)
      for (int e = 0; e < nj; e++) {
        ni_out[o_] = T.first_child[i] + c;
        nj_out[o_] = T.first_child[j] + e;
        o_++;
      }
  } else if (ni == 0) {
    for (int e = 0; e < nj; e++) {
      ni_out[o_] = i;
      nj_out[o_] = T.first_child[j] + e;
      o_++;
    }
  } else {
    for (int c = 0; c < ni; c++) {
      ni_out[o_] = T.first_child[i] + c;
      nj_out[o_] = j;
      o_++;
    }
  }
}

// Sorting a pair list by (i, j): count per row i, scan, scatter the j's
// into their row (any order), then sort each row's j's (rows are short: the
// pairs of one node) and write i and the CSR row pointer.
__global__ void k_row_hist(const int *pi, int64_t n, int *rc) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a < n) atomicAdd(&rc[pi[a]], 1);
}

__global__ void k_row_widen(const int *rc, int nnodes, int64_t *out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nnodes) out[i] = rc[i];
}

__global__ void k_row_scatter(const int *pi, const int *pj, int64_t n, const int64_t *ro,
                              int *fill, int *sj) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const int i = pi[a];
  sj[ro[i] + atomicAdd(&fill[i], 1)] = pj[a];
}

// one workgroup per row: a j's position in its sorted row is the number of
// the row's entries that precede it in (j, scatter position) order, counted
// from a copy of the row in LDS; rows longer than RK_MAX (not produced by
// the separation test with tau < 1 in d <= 3) are sorted by one thread
constexpr int RK_MAX = 2048;
__global__ void __launch_bounds__(64) k_row_sort(const int64_t *ro, int nnodes, const int *sj_in,
                                                 int *si, int *sj, int *row) {
  __shared__ int v[RK_MAX];
  const int i = blockIdx.x, t = threadIdx.x;
  if (t == 0) {
    row[i] = (int)ro[i];
    if (i == nnodes - 1) row[nnodes] = (int)ro[nnodes];
  }
  const int64_t b = ro[i], e = ro[i + 1];
  const int r = (int)(e - b);
  if (r <= RK_MAX) {
    for (int a = t; a < r; a += 64) v[a] = sj_in[b + a];
    __syncthreads();
    for (int a = t; a < r; a += 64) {
      const int x = v[a];
      int cnt = 0;
      for (int c = 0; c < r; c++) {
        const int y = v[c];
        cnt += (y < x || (y == x && c < a)) ? 1 : 0;
      }
      sj[b + cnt] = x;
      si[b + cnt] = i;
    }
  } else if (t == 0) {
    for (int64_t a = b; a < e; a++) sj[a] = sj_in[a];
    for (int64_t a = b + 1; a < e; a++) {
      const int x = sj[a];
      int64_t c = a - 1;
      while (c >= b && sj[c] > x) {
        sj[c + 1] = sj[c];
        c--;
      }
      sj[c + 1] = x;
    }
    for (int64_t a = b; a < e; a++) si[a] = i;
  }
}

// CSR row pointer of a list sorted by i: row[i] = first entry with key >= i
__global__ void k_csr_rows(const int *pi, int64_t n, int nnodes, int *row) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > nnodes) return;
  int64_t b = 0, e = n;
  while (b < e) {
    int64_t m = b + (e - b) / 2;
    if (pi[m] < i)
      b = m + 1;
    else
      e = m;
  }
  row[i] = (int)b;
}

// ---- HSS (3.5): siblings and diagonal leaves
__global__ void k_hss_count(TreeView T, int nnodes, int64_t *cL, int64_t *cLm) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnodes) return;
  cL[i] = i == 0 ? 0 : T.nchild[T.parent[i]] - 1;
  cLm[i] = T.nchild[i] == 0 ? 1 : 0;
}

__global__ void k_hss_emit(TreeView T, int nnodes, const int64_t *oL, const int64_t *oLm, int *Li,
                           int *Lj, int *Lmi, int *Lmj) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnodes) return;
  if (i > 0) {
    int p = T.parent[i];
    int64_t o = oL[i];
    for (int c = 0; c < T.nchild[p]; c++) {
      int s = T.first_child[p] + c;
      if (s != i) {
        Li[o] = i;
        Lj[o] = s;
        o++;
      }
    }
  }
  if (T.nchild[i] == 0) {
    Lmi[oLm[i]] = i;
    Lmj[oLm[i]] = i;
  }
}

// ---- HSS near-field sets (A.1), one level at a time, top-down
__global__ void k_near_count(TreeView T, int nb, int ne, const int *Nrow, const int *Ncol, int d,
                             double tau, int64_t *cnt) {
  int i = nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  int p = T.parent[i];
  int64_t c = T.nchild[p] - 1;
  for (int a = Nrow[p]; a < Nrow[p + 1]; a++) {
    int m = Ncol[a];
    if (T.nchild[m] == 0) {
      if (!well_separated(T.lo, T.hi, i, m, d, tau)) c++;
    } else {
      for (int q = 0; q < T.nchild[m]; q++)
        if (!well_separated(T.lo, T.hi, i, T.first_child[m] + q, d, tau)) c++;
    }
  }
  cnt[i - nb] = c;
}

__global__ void k_near_emit(TreeView T, int nb, int ne, int *Nrow, int *Ncol, const int64_t *off,
                            int d, double tau) {
  int i = nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  int p = T.parent[i];
  int64_t o = off[i - nb];
  Nrow[i] = (int)o;
  for (int c = 0; c < T.nchild[p]; c++) {
    int s = T.first_child[p] + c;
    if (s != i) Ncol[o++] = s;
  }
  for (int a = Nrow[p]; a < Nrow[p + 1]; a++) {
    int m = Ncol[a];
    if (T.nchild[m] == 0) {
      if (!well_separated(T.lo, T.hi, i, m, d, tau)) Ncol[o++] = m;
    } else {
      for (int q = 0; q < T.nchild[m]; q++) {
        int k = T.first_child[m] + q;
        if (!well_separated(T.lo, T.hi, i, k, d, tau)) Ncol[o++] = k;
      }
    }
  }
  if (i == ne - 1) Nrow[ne] = (int)off[ne - nb];
}

template <class T>
static T readback1(hipStream_t s, const T *dev) {
  return read_one(s, dev);
}

// the n pairs (pi, pj) sorted by (i, j) into handle memory, with the CSR
// row pointer (nnodes + 1 entries)
static void sort_pairs_by_row(Handle &h, const int *pi, const int *pj, int64_t n, int *&oi,
                              int *&oj, int *&row, DeviceArena &tmp) {
  hipStream_t s = h.stream;
  const int nn = (int)h.nnodes;
  oi = h.mem.alloc_n<int>(n);
  oj = h.mem.alloc_n<int>(n);
  row = h.mem.alloc_n<int>(nn + 1);
  int *rc = tmp.alloc_n<int>(2 * (int64_t)nn);
  int *fill = rc + nn;
  int64_t *rc64 = tmp.alloc_n<int64_t>(nn), *ro = tmp.alloc_n<int64_t>(nn + 1);
  SMASH_HIP(hipMemsetAsync(rc, 0, sizeof(int) * 2 * (size_t)nn, s));
  if (n > 0) {
    k_row_hist<<<ceil_div(n, 256), 256, 0, s>>>(pi, n, rc);
    SMASH_CHECK_LAUNCH();
  }
  k_row_widen<<<ceil_div(nn, 256), 256, 0, s>>>(rc, nn, rc64);
  SMASH_CHECK_LAUNCH();
  scan_i64(rc64, ro, nn, nullptr, s, tmp);
  int *sc = tmp.alloc_n<int>(n > 0 ? n : 1);
  if (n > 0) {
    k_row_scatter<<<ceil_div(n, 256), 256, 0, s>>>(pi, pj, n, ro, fill, sc);
    SMASH_CHECK_LAUNCH();
  }
  k_row_sort<<<nn, 64, 0, s>>>(ro, nn, sc, oi, oj, row);
  SMASH_CHECK_LAUNCH();
}

// grows a pair buffer (i and j arrays) to hold `need` entries, keeping the
// first `used`
static void grow_pairs(int *&bi, int *&bj, int64_t &cap, int64_t used, int64_t need,
                       DeviceArena &tmp, hipStream_t s) {
  if (need <= cap) return;
  int64_t nc = cap > 0 ? cap : 1024;
  while (nc < need) nc *= 2;
  int *ni = tmp.alloc_n<int>(nc), *nj = tmp.alloc_n<int>(nc);
  if (used > 0) {
    SMASH_HIP(hipMemcpyAsync(ni, bi, sizeof(int) * used, hipMemcpyDeviceToDevice, s));
    SMASH_HIP(hipMemcpyAsync(nj, bj, sizeof(int) * used, hipMemcpyDeviceToDevice, s));
  }
  bi = ni;
  bj = nj;
  cap = nc;
}

void build_pairs(Handle &h) {
  hipStream_t s = h.stream;
  DeviceArena tmp;
  tmp.stream = s;
  TreeView T = view(h);
  try {
    if (h.adm == SMASH_ADM_STRONG) {
      // frontier expansion; L and L^- pairs appended to growing buffers
      int *Lbi = nullptr, *Lbj = nullptr, *Mbi = nullptr, *Mbj = nullptr;
      int64_t capL = 0, capM = 0, nLacc = 0, nMacc = 0;
      grow_pairs(Lbi, Lbj, capL, 0, 32 * h.nnodes + 1024, tmp, s);
      grow_pairs(Mbi, Mbj, capM, 0, 8 * h.nnodes + 1024, tmp, s);
      int *fi = tmp.alloc_n<int>(1), *fj = tmp.alloc_n<int>(1);
      SMASH_HIP(hipMemsetAsync(fi, 0, sizeof(int), s));
      SMASH_HIP(hipMemsetAsync(fj, 0, sizeof(int), s));
      int64_t nf = 1;
      while (nf > 0) {
        int64_t *c = tmp.alloc_n<int64_t>(3 * nf), *o = tmp.alloc_n<int64_t>(3 * nf + 1);
        k_front_count<<<ceil_div(nf, 256), 256, 0, s>>>(T, fi, fj, nf, h.d, h.tau, c, c + nf,
                                                        c + 2 * nf);
        SMASH_CHECK_LAUNCH();
        scan_i64(c, o, 3 * nf, nullptr, s, tmp);
        const int64_t *pin = pick_words(s, {{o + nf, 8}, {o + 2 * nf, 8}, {o + 3 * nf, 8}});
        const int64_t tL = pin[0], tLm = pin[1], tE = pin[2];
        const int64_t nLg = tL, nMg = tLm - tL, nEg = tE - tLm;
        grow_pairs(Lbi, Lbj, capL, nLacc, nLacc + nLg, tmp, s);
        grow_pairs(Mbi, Mbj, capM, nMacc, nMacc + nMg, tmp, s);
        int *ni = tmp.alloc_n<int>(nEg), *nj = tmp.alloc_n<int>(nEg);
        k_front_emit<<<ceil_div(nf, 256), 256, 0, s>>>(T, fi, fj, nf, o, tL, tLm, Lbi + nLacc,
                                                       Lbj + nLacc, Mbi + nMacc, Mbj + nMacc,
                                                       ni, nj);
        SMASH_CHECK_LAUNCH();
        nLacc += nLg;
        nMacc += nMg;
        fi = ni;
        fj = nj;
        nf = nEg;
      }
      h.nL = nLacc;
      h.nLm = nMacc;
      sort_pairs_by_row(h, Lbi, Lbj, h.nL, h.Li, h.Lj, h.Lrow, tmp);
      sort_pairs_by_row(h, Mbi, Mbj, h.nLm, h.Lmi, h.Lmj, h.Lmrow, tmp);
    } else {
      int nn = h.nnodes;
      int64_t *c = tmp.alloc_n<int64_t>(2 * nn), *o = tmp.alloc_n<int64_t>(2 * (nn + 1));
      k_hss_count<<<ceil_div(nn, 256), 256, 0, s>>>(T, nn, c, c + nn);
      SMASH_CHECK_LAUNCH();
      scan_i64(c, o, nn, nullptr, s, tmp);
      scan_i64(c + nn, o + nn + 1, nn, nullptr, s, tmp);
      h.nL = readback1(s, o + nn);
      h.nLm = readback1(s, o + 2 * nn + 1);
      h.Li = h.mem.alloc_n<int>(h.nL);
      h.Lj = h.mem.alloc_n<int>(h.nL);
      h.Lmi = h.mem.alloc_n<int>(h.nLm);
      h.Lmj = h.mem.alloc_n<int>(h.nLm);
      k_hss_emit<<<ceil_div(nn, 256), 256, 0, s>>>(T, nn, o, o + nn + 1, h.Li, h.Lj, h.Lmi, h.Lmj);
      SMASH_CHECK_LAUNCH();
      // near-field sets, level by level (root: empty)
      h.Nrow = h.mem.alloc_n<int>(nn + 1);
      SMASH_HIP(hipMemsetAsync(h.Nrow, 0, sizeof(int) * 2, s));
      int64_t cap = 4 * (int64_t)nn + 16, used = 0;
      h.Ncol = h.mem.alloc_n<int>(cap);
      for (int l = 2; l <= h.nlevels; l++) {
        int nb = h.level_beg[l - 1], ne = h.level_beg[l];
        int64_t *cnt = tmp.alloc_n<int64_t>(ne - nb), *off = tmp.alloc_n<int64_t>(ne - nb + 1);
        int64_t *base = tmp.alloc_n<int64_t>(1);
        set_i64(base, used, s);
        k_near_count<<<ceil_div(ne - nb, 256), 256, 0, s>>>(T, nb, ne, h.Nrow, h.Ncol, h.d, h.tau,
                                                            cnt);
        SMASH_CHECK_LAUNCH();
        scan_i64(cnt, off, ne - nb, base, s, tmp);
        int64_t nu = readback1(s, off + (ne - nb));
        if (nu > cap) {
          int64_t nc = cap;
          while (nc < nu) nc *= 2;
          int *q = h.mem.alloc_n<int>(nc);
          SMASH_HIP(hipMemcpyAsync(q, h.Ncol, sizeof(int) * used, hipMemcpyDeviceToDevice, s));
          h.Ncol = q;
          cap = nc;
        }
        k_near_emit<<<ceil_div(ne - nb, 256), 256, 0, s>>>(T, nb, ne, h.Nrow, h.Ncol, off, h.d,
                                                           h.tau);
        SMASH_CHECK_LAUNCH();
        used = nu;
      }
      h.nN = used;
    }
    if (h.adm != SMASH_ADM_STRONG) {
      h.Lrow = h.mem.alloc_n<int>(h.nnodes + 1);
      h.Lmrow = h.mem.alloc_n<int>(h.nnodes + 1);
      k_csr_rows<<<ceil_div(h.nnodes + 1, 256), 256, 0, s>>>(h.Li, h.nL, h.nnodes, h.Lrow);
      SMASH_CHECK_LAUNCH();
      k_csr_rows<<<ceil_div(h.nnodes + 1, 256), 256, 0, s>>>(h.Lmi, h.nLm, h.nnodes, h.Lmrow);
      SMASH_CHECK_LAUNCH();
    }
    defer_release(h, tmp);
  } catch (...) {
    (void)hipStreamSynchronize(s);
    tmp.release();
    throw;
  }
}

}  // namespace smash
