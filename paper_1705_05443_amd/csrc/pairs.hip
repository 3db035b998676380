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

__global__ void k_front_emit(TreeView T, const int *fi, const int *fj, int64_t nf,
                             const int64_t *oL, const int64_t *oLm, const int64_t *oE, int *Li,
                             int *Lj, int *Lmi, int *Lmj, int *ni_out, int *nj_out) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int i = fi[f], j = fj[f];
  if (oL[f + 1] > oL[f]) {
    Li[oL[f]] = i;
    Lj[oL[f]] = j;
    return;
  }
  if (oLm[f + 1] > oLm[f]) {
    Lmi[oLm[f]] = i;
    Lmj[oLm[f]] = j;
    return;
  }
  int64_t o = oE[f];
  int ni = T.nchild[i], nj = T.nchild[j];
  if (ni > 0 && nj > 0) {
    for (int c = 0; c < ni; c++)
      for (int e = 0; e < nj; e++) {
        ni_out[o] = T.first_child[i] + c;
        nj_out[o] = T.first_child[j] + e;
        o++;
      }
  } else if (ni == 0) {
    for (int e = 0; e < nj; e++) {
      ni_out[o] = i;
      nj_out[o] = T.first_child[j] + e;
      o++;
    }
  } else {
    for (int c = 0; c < ni; c++) {
      ni_out[o] = T.first_child[i] + c;
      nj_out[o] = j;
      o++;
    }
  }
}

__global__ void k_pair_keys(const int *pi, const int *pj, int64_t n, int nnodes, uint64_t *keys,
                            int32_t *vals) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  keys[a] = (uint64_t)pi[a] * (uint64_t)nnodes + (uint64_t)pj[a];
  vals[a] = (int32_t)a;
}

__global__ void k_pair_unkey(const uint64_t *keys, int64_t n, int nnodes, int *pi, int *pj) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  pi[a] = (int)(keys[a] / (uint64_t)nnodes);
  pj[a] = (int)(keys[a] % (uint64_t)nnodes);
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

static int bits_for(uint64_t v) {
  int b = 0;
  while (b < 64 && (v >> b) != 0) b++;
  return b;
}

static void sort_pairs(Handle &h, int *&pi, int *&pj, int64_t n, DeviceArena &tmp) {
  hipStream_t s = h.stream;
  int *oi = h.mem.alloc_n<int>(n), *oj = h.mem.alloc_n<int>(n);
  if (n > 0) {
    uint64_t *k1 = tmp.alloc_n<uint64_t>(n), *k2 = tmp.alloc_n<uint64_t>(n);
    int32_t *v1 = tmp.alloc_n<int32_t>(n), *v2 = tmp.alloc_n<int32_t>(n);
    k_pair_keys<<<ceil_div(n, 256), 256, 0, s>>>(pi, pj, n, h.nnodes, k1, v1);
    SMASH_CHECK_LAUNCH();
    int nb = bits_for((uint64_t)h.nnodes * (uint64_t)h.nnodes);
    radix_sort_u64(k1, v1, k2, v2, n, nb, s, tmp);
    k_pair_unkey<<<ceil_div(n, 256), 256, 0, s>>>(k1, n, h.nnodes, oi, oj);
    SMASH_CHECK_LAUNCH();
  }
  pi = oi;
  pj = oj;
}

void build_pairs(Handle &h) {
  hipStream_t s = h.stream;
  DeviceArena tmp;
  tmp.stream = s;
  TreeView T = view(h);
  try {
    if (h.adm == SMASH_ADM_STRONG) {
      // frontier expansion
      std::vector<int *> Lis, Ljs, Lmis, Lmjs;
      std::vector<int64_t> Lns, Lmns;
      int *fi = tmp.alloc_n<int>(1), *fj = tmp.alloc_n<int>(1);
      SMASH_HIP(hipMemsetAsync(fi, 0, sizeof(int), s));
      SMASH_HIP(hipMemsetAsync(fj, 0, sizeof(int), s));
      int64_t nf = 1;
      while (nf > 0) {
        int64_t *c = tmp.alloc_n<int64_t>(3 * nf), *o = tmp.alloc_n<int64_t>(3 * (nf + 1));
        k_front_count<<<ceil_div(nf, 256), 256, 0, s>>>(T, fi, fj, nf, h.d, h.tau, c, c + nf,
                                                        c + 2 * nf);
        SMASH_CHECK_LAUNCH();
        scan_i64(c, o, nf, nullptr, s, tmp);
        scan_i64(c + nf, o + nf + 1, nf, nullptr, s, tmp);
        scan_i64(c + 2 * nf, o + 2 * (nf + 1), nf, nullptr, s, tmp);
        const int64_t *pin = pick_words(s, {{o + nf, 8}, {o + 2 * nf + 1, 8}, {o + 3 * nf + 2, 8}});
        const int64_t tot[3] = {pin[0], pin[1], pin[2]};
        int *li = tmp.alloc_n<int>(tot[0]), *lj = tmp.alloc_n<int>(tot[0]);
        int *mi = tmp.alloc_n<int>(tot[1]), *mj = tmp.alloc_n<int>(tot[1]);
        int *ni = tmp.alloc_n<int>(tot[2]), *nj = tmp.alloc_n<int>(tot[2]);
        k_front_emit<<<ceil_div(nf, 256), 256, 0, s>>>(T, fi, fj, nf, o, o + nf + 1,
                                                       o + 2 * (nf + 1), li, lj, mi, mj, ni, nj);
        SMASH_CHECK_LAUNCH();
        Lis.push_back(li);
        Ljs.push_back(lj);
        Lns.push_back(tot[0]);
        Lmis.push_back(mi);
        Lmjs.push_back(mj);
        Lmns.push_back(tot[1]);
        fi = ni;
        fj = nj;
        nf = tot[2];
      }
      // concatenate the generations, then sort
      auto concat = [&](std::vector<int *> &a, std::vector<int *> &b, std::vector<int64_t> &n,
                        int *&oi, int *&oj) -> int64_t {
        int64_t tot = 0;
        for (auto v : n) tot += v;
        oi = tmp.alloc_n<int>(tot);
        oj = tmp.alloc_n<int>(tot);
        int64_t o = 0;
        for (size_t g = 0; g < n.size(); g++) {
          if (n[g] == 0) continue;
          SMASH_HIP(hipMemcpyAsync(oi + o, a[g], sizeof(int) * n[g], hipMemcpyDeviceToDevice, s));
          SMASH_HIP(hipMemcpyAsync(oj + o, b[g], sizeof(int) * n[g], hipMemcpyDeviceToDevice, s));
          o += n[g];
        }
        return tot;
      };
      int *ai, *aj, *bi, *bj;
      h.nL = concat(Lis, Ljs, Lns, ai, aj);
      h.nLm = concat(Lmis, Lmjs, Lmns, bi, bj);
      sort_pairs(h, ai, aj, h.nL, tmp);
      sort_pairs(h, bi, bj, h.nLm, tmp);
      h.Li = ai;
      h.Lj = aj;
      h.Lmi = bi;
      h.Lmj = bj;
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
    h.Lrow = h.mem.alloc_n<int>(h.nnodes + 1);
    h.Lmrow = h.mem.alloc_n<int>(h.nnodes + 1);
    k_csr_rows<<<ceil_div(h.nnodes + 1, 256), 256, 0, s>>>(h.Li, h.nL, h.nnodes, h.Lrow);
    SMASH_CHECK_LAUNCH();
    k_csr_rows<<<ceil_div(h.nnodes + 1, 256), 256, 0, s>>>(h.Lmi, h.nLm, h.nnodes, h.Lmrow);
    SMASH_CHECK_LAUNCH();
    SMASH_HIP(hipStreamSynchronize(s));
    tmp.release();
  } catch (...) {
    (void)hipStreamSynchronize(s);
    tmp.release();
    throw;
  }
}

}  // namespace smash
