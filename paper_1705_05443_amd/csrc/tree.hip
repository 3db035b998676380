// tree.hip -- adaptive partition of Sec. 3.1 (binary bisection for HSS,
// Remark A.1) and the point permutation.
//
// Every point gets its full bisection key: the sequence of half-box choices
// (x >= mid goes up, mid = 0.5*(lo+hi)) from the root box down through all
// bisection stages the 64-bit key allows, most significant first, axis 0
// first inside a stage.  A stable radix sort by key gives the permutation:
// every box of the tree is then a contiguous range, and inside a leaf the
// points keep the order of their finer bisection path (ties: input order).
// Nodes are then discovered level by level: a node holding more than nu_0
// points of X or of Y is split into its non-empty children, whose ranges
// are found by binary searches on the key digit of that stage (one thread
// per child boundary, all boundaries of a level at once).
#include "common.cuh"

namespace smash {

struct Geom {
  double lo[3], hi[3];
  int d, hss, bpl, max_split;
  int split_cap;  // bisection stages the keys are sorted by (<= max_split)
};

__global__ void k_keys(const double *__restrict__ pts, int64_t n, Geom g,
                       uint64_t *__restrict__ keys, int32_t *__restrict__ idx) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double x[3], lo[3], hi[3];
  for (int t = 0; t < g.d; t++) {
    x[t] = pts[a * g.d + t];
    lo[t] = g.lo[t];
    hi[t] = g.hi[t];
  }
  uint64_t key = 0;
  for (int s = 0; s < g.max_split; s++) {
    for (int u = 0; u < g.bpl; u++) {
      int t = g.hss ? (s % g.d) : u;
      double mid = 0.5 * (lo[t] + hi[t]);
      bool up = x[t] >= mid;
      key = (key << 1) | (uint64_t)up;
      if (up)
        lo[t] = mid;
      else
        hi[t] = mid;
    }
  }
  keys[a] = key;
  idx[a] = (int32_t)a;
}

__global__ void k_gather_points(const double *__restrict__ pts, const int32_t *__restrict__ perm,
                                int64_t n, int d, double *__restrict__ out) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  int64_t src = perm[a];
  for (int t = 0; t < d; t++) out[a * d + t] = pts[src * d + t];
}

__device__ inline int key_digit(uint64_t key, int s, const Geom &g) {
  int shift = (g.max_split - 1 - s) * g.bpl;
  return (int)((key >> shift) & ((1ull << g.bpl) - 1ull));
}

// first index in [b, e) whose stage-s digit exceeds v (digits ascend there)
__device__ inline int run_end(const uint64_t *keys, int b, int e, int s, int v, const Geom &g) {
  while (b < e) {
    int mid = b + (e - b) / 2;
    if (key_digit(keys[mid], s, g) <= v)
      b = mid + 1;
    else
      e = mid;
  }
  return b;
}

struct NodeArrays {
  int *level, *parent, *first_child, *nchild, *xb, *xe, *yb, *ye;
  double *lo, *hi;
};

// Child boundaries of every splitting node of a level, all searched at once:
// thread (node, side, v) finds the first index of the node's range whose
// stage-s digit exceeds v (v < 2^bpl - 1; the last child ends at the range
// end).  bnd holds nsides * (2^bpl - 1) entries per node of the level.
__global__ void k_tree_bounds(NodeArrays N, int nb, int ne, const uint64_t *kx,
                              const uint64_t *ky, int s, int leaf, Geom g, int nsides, int *bnd) {
  const int nv = (1 << g.bpl) - 1;
  const int per = nsides * nv;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)(ne - nb) * per) return;
  const int i = nb + (int)(t / per), r = (int)(t % per), side = r / nv, v = r % nv;
  const int xb = N.xb[i], xe = N.xe[i], yb = N.yb[i], ye = N.ye[i];
  const bool split = (xe - xb > leaf || ye - yb > leaf) && s < g.split_cap;
  if (!split) return;
  bnd[t] = side ? run_end(ky, yb, ye, s, v, g) : run_end(kx, xb, xe, s, v, g);
}

// end of child v's X (side 0) or Y range from the searched boundaries
__device__ inline int child_end(const int *bn, int nsides, int nv, int side, int v, int e) {
  return v < nv ? bn[(nsides > 1 ? side : 0) * nv + v] : e;
}

__global__ void k_tree_split(NodeArrays N, int nb, int ne, int s, int leaf, Geom g, int nsides,
                             const int *bnd, int64_t *cnt, int *deeper) {
  int i = nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  int xb = N.xb[i], xe = N.xe[i], yb = N.yb[i], ye = N.ye[i];
  bool split = (xe - xb > leaf || ye - yb > leaf) && s < g.split_cap;
  // a node that needs the stages the keys were not sorted by
  if ((xe - xb > leaf || ye - yb > leaf) && s >= g.split_cap && g.split_cap < g.max_split)
    atomicOr(deeper, 1);
  int c = 0;
  if (split) {
    const int nv = (1 << g.bpl) - 1;
    const int *bn = bnd + (int64_t)(i - nb) * nsides * nv;
    int ax = xb, ay = yb;
    for (int v = 0; v <= nv; v++) {
      int bx = child_end(bn, nsides, nv, 0, v, xe), by = child_end(bn, nsides, nv, 1, v, ye);
      if (bx > ax || by > ay) c++;
      ax = bx;
      ay = by;
    }
  }
  cnt[i - nb] = c;
}

__global__ void k_tree_emit(NodeArrays N, int nb, int ne, int s, int leaf, Geom g, int nsides,
                            const int *bnd, const int64_t *off) {
  int i = nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  int xb = N.xb[i], xe = N.xe[i], yb = N.yb[i], ye = N.ye[i];
  bool split = (xe - xb > leaf || ye - yb > leaf) && s < g.split_cap;
  int first = (int)off[i - nb];
  int c = 0;
  if (split) {
    const int nv = (1 << g.bpl) - 1;
    const int *bn = bnd + (int64_t)(i - nb) * nsides * nv;
    int ax = xb, ay = yb;
    for (int v = 0; v <= nv; v++) {
      int bx = child_end(bn, nsides, nv, 0, v, xe), by = child_end(bn, nsides, nv, 1, v, ye);
      if (bx > ax || by > ay) {
        int ch = first + c;
        N.level[ch] = N.level[i] + 1;
        N.parent[ch] = i;
        N.first_child[ch] = -1;
        N.nchild[ch] = 0;
        N.xb[ch] = ax;
        N.xe[ch] = bx;
        N.yb[ch] = ay;
        N.ye[ch] = by;
        for (int t = 0; t < 3; t++) {
          N.lo[3 * ch + t] = N.lo[3 * i + t];
          N.hi[3 * ch + t] = N.hi[3 * i + t];
        }
        for (int u = 0; u < g.bpl; u++) {
          int t = g.hss ? (s % g.d) : u;
          int up = (v >> (g.bpl - 1 - u)) & 1;
          double mid = 0.5 * (N.lo[3 * i + t] + N.hi[3 * i + t]);
          if (up)
            N.lo[3 * ch + t] = mid;
          else
            N.hi[3 * ch + t] = mid;
        }
        c++;
      }
      ax = bx;
      ay = by;
    }
  }
  N.nchild[i] = c;
  N.first_child[i] = c > 0 ? first : -1;
}

// Points of one leaf in the order of their full keys, ties by input index
// (what one stable sort of the full keys gives), when the keys were sorted
// only by the leading stages: one workgroup per leaf, the leaf's keys and
// indices in LDS, each point's position = the number of points before it.
constexpr int LS_MAX = 1024;
__global__ void __launch_bounds__(64) k_leaf_sort(const int *nchild, const int *b32,
                                                  const int *e32, int nnodes, uint64_t *keys,
                                                  int *perm) {
  __shared__ uint64_t kk[LS_MAX];
  __shared__ int pp[LS_MAX];
  const int i = blockIdx.x, t = threadIdx.x;
  if (i >= nnodes || nchild[i] != 0) return;
  const int b = b32[i], r = e32[i] - b;
  if (r <= 1 || r > LS_MAX) return;  // (the caller guarantees r <= LS_MAX)
  for (int a = t; a < r; a += 64) {
    kk[a] = keys[b + a];
    pp[a] = perm[b + a];
  }
  __syncthreads();
  for (int a = t; a < r; a += 64) {
    const uint64_t x = kk[a];
    const int px = pp[a];
    int cnt = 0;
    for (int c = 0; c < r; c++) {
      const uint64_t y = kk[c];
      cnt += (y < x || (y == x && pp[c] < px)) ? 1 : 0;
    }
    keys[b + cnt] = x;
    perm[b + cnt] = px;
  }
}

__global__ void k_root(NodeArrays N, int nx, int ny, Geom g) {
  N.level[0] = 1;
  N.parent[0] = -1;
  N.first_child[0] = -1;
  N.nchild[0] = 0;
  N.xb[0] = 0;
  N.xe[0] = nx;
  N.yb[0] = 0;
  N.ye[0] = ny;
  for (int t = 0; t < 3; t++) {
    N.lo[t] = t < g.d ? g.lo[t] : 0.0;
    N.hi[t] = t < g.d ? g.hi[t] : 0.0;
  }
}

// min / max of one coordinate over a point set (root bounding cube)
__global__ void k_minmax(const double *pts, int64_t n, int d, double *out /* 2*d */) {
  __shared__ double smin[256], smax[256];
  for (int t = 0; t < d; t++) {
    double mn = INFINITY, mx = -INFINITY;
    for (int64_t a = threadIdx.x; a < n; a += blockDim.x) {
      double v = pts[a * d + t];
      mn = fmin(mn, v);
      mx = fmax(mx, v);
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) {
        smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
        smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      out[2 * t] = smin[0];
      out[2 * t + 1] = smax[0];
    }
    __syncthreads();
  }
}

// counts of non-finite coordinates and of coordinates outside [lo, hi]
__global__ void k_check_points(const double *pts, int64_t n, int d, Geom g, int use_box,
                               int *bad) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  for (int t = 0; t < d; t++) {
    double v = pts[a * d + t];
    if (!isfinite(v)) atomicOr(&bad[0], 1);
    if (use_box && !(v >= g.lo[t] && v <= g.hi[t])) atomicOr(&bad[1], 1);
  }
}

static void grow_nodes(Handle &h, int &cap, int need) {
  if (need <= cap) return;
  int nc = cap > 0 ? cap : 1024;
  while (nc < need) nc *= 2;
  auto regrow_i = [&](int *&p) {
    int *q = h.mem.alloc_n<int>(nc);
    if (p) SMASH_HIP(hipMemcpyAsync(q, p, sizeof(int) * cap, hipMemcpyDeviceToDevice, h.stream));
    p = q;
  };
  auto regrow_d = [&](double *&p) {
    double *q = h.mem.alloc_n<double>(3 * (size_t)nc);
    if (p)
      SMASH_HIP(hipMemcpyAsync(q, p, sizeof(double) * 3 * cap, hipMemcpyDeviceToDevice, h.stream));
    p = q;
  };
  regrow_i(h.level);
  regrow_i(h.parent);
  regrow_i(h.first_child);
  regrow_i(h.nchild);
  regrow_i(h.xb);
  regrow_i(h.xe);
  regrow_i(h.yb);
  regrow_i(h.ye);
  regrow_d(h.lo);
  regrow_d(h.hi);
  cap = nc;
}

template <class T>
static T readback(Handle &h, const T *dev) {
  return read_one(h.stream, dev);
}

void build_tree(Handle &h, const double *x, const double *y) {
  hipStream_t s = h.stream;
  DeviceArena tmp;
  tmp.stream = s;
  try {
    Geom g;
    g.d = h.d;
    g.hss = h.adm == SMASH_ADM_WEAK;
    g.bpl = h.bpl;
    g.max_split = h.max_split;
    g.split_cap = h.max_split;
    for (int t = 0; t < 3; t++) {
      g.lo[t] = h.root_lo[t];
      g.hi[t] = h.root_hi[t];
    }
    // validate the points (and compute the bounding cube if no root box)
    int *bad = tmp.alloc_n<int>(2);
    SMASH_HIP(hipMemsetAsync(bad, 0, 2 * sizeof(int), s));
    // finite coordinates everywhere; inside the root box when one is given
    const int use_box = h.has_root ? 1 : 0;
    k_check_points<<<ceil_div(h.nx, 256), 256, 0, s>>>(x, h.nx, h.d, g, use_box, bad);
    SMASH_CHECK_LAUNCH();
    if (!h.same_xy) {
      k_check_points<<<ceil_div(h.ny, 256), 256, 0, s>>>(y, h.ny, h.d, g, use_box, bad);
      SMASH_CHECK_LAUNCH();
    }
    // one read of the flags (and of the bounding box without a root box)
    int64_t *pin = pinned_words();
    double *mm = nullptr;
    if (!h.has_root) {
      mm = tmp.alloc_n<double>(12);
      k_minmax<<<1, 256, 0, s>>>(x, h.nx, h.d, mm);
      SMASH_CHECK_LAUNCH();
      k_minmax<<<1, 256, 0, s>>>(y, h.ny, h.d, mm + 6);
      SMASH_CHECK_LAUNCH();
      SMASH_HIP(hipMemcpyAsync(pin + 2, mm, 12 * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    SMASH_HIP(hipMemcpyAsync(pin, bad, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    stream_wait(s);
    int hb[2];
    std::memcpy(hb, pin, sizeof(hb));
    if (hb[0]) throw Error{SMASH_E_NUMERIC, "non-finite point coordinate"};
    if (h.has_root && hb[1]) throw Error{SMASH_E_INVALID_ARG, "a point lies outside the root box"};
    if (!h.has_root) {
      // bounding cube of X and Y: lo = min, side = largest extent
      double hm[12];
      std::memcpy(hm, pin + 2, sizeof(hm));
      double side = 0.0;
      for (int t = 0; t < h.d; t++) {
        double mn = hm[2 * t] < hm[6 + 2 * t] ? hm[2 * t] : hm[6 + 2 * t];
        double mx = hm[2 * t + 1] > hm[6 + 2 * t + 1] ? hm[2 * t + 1] : hm[6 + 2 * t + 1];
        h.root_lo[t] = mn;
        if (mx - mn > side) side = mx - mn;
      }
      for (int t = 0; t < h.d; t++) h.root_hi[t] = h.root_lo[t] + side;
      for (int t = 0; t < 3; t++) {
        g.lo[t] = h.root_lo[t];
        g.hi[t] = h.root_hi[t];
      }
    }
    tmp.release();

    // Keys and stable sort (X, then Y unless Y is X).  First by the leading
    // stages only (at most 24 key bits); if the tree needs no deeper stage,
    // each leaf is then put in full-key order by itself, which gives the
    // permutation of a full sort.  Otherwise the keys are sorted in full and
    // the tree is rebuilt.
    int keybits = g.max_split * g.bpl;
    uint64_t *kx = nullptr, *ky = nullptr;
    int32_t *px = nullptr, *py = nullptr;
    auto make_keys = [&](const double *pts, int64_t n, uint64_t *&k, int32_t *&perm) {
      k = tmp.alloc_n<uint64_t>(n);
      perm = h.mem.alloc_n<int>(n);
      k_keys<<<ceil_div(n, 256), 256, 0, s>>>(pts, n, g, k, perm);
      SMASH_CHECK_LAUNCH();
    };
    auto sort_keys = [&](uint64_t *k, int32_t *perm, int64_t n, int lo_bit) {
      uint64_t *k2 = tmp.alloc_n<uint64_t>(n);
      int32_t *v2 = tmp.alloc_n<int32_t>(n);
      radix_sort_u64(k, perm, k2, v2, n, keybits, s, tmp, lo_bit);
    };
    int *deeper = tmp.alloc_n<int>(1);
    // first capacity from the usual node count (a tree of n points in
    // leaves of at most `leaf` holds about 2.5 n / leaf nodes), so that
    // regrowth (a copy of every node array) is the exception
    int cap = 0;
    {
      const int64_t np = std::max(h.nx, h.ny);
      const int64_t guess = 4 * (np / std::max(1, h.leaf) + 1) * (h.bpl > 1 ? 2 : 1);
      grow_nodes(h, cap, (int)std::min<int64_t>(std::max<int64_t>(1024, guess), 1 << 24));
    }
    NodeArrays N;
    auto refresh = [&]() {
      N = NodeArrays{h.level, h.parent, h.first_child, h.nchild, h.xb, h.xe, h.yb, h.ye,
                     h.lo, h.hi};
    };
    int nb = 0, ne = 1, lev = 1;
    // nodes, level by level; returns whether a node needs stages beyond split_cap
    auto grow_tree = [&]() -> bool {
      refresh();
      SMASH_HIP(hipMemsetAsync(deeper, 0, sizeof(int), s));
      k_root<<<1, 1, 0, s>>>(N, (int)h.nx, (int)h.ny, g);
      SMASH_CHECK_LAUNCH();
      h.level_beg.assign(1, 0);
      nb = 0;
      ne = 1;
      lev = 1;
      for (;;) {
        h.level_beg.push_back(ne);
        int cnt_n = ne - nb;
        int64_t *cnt = tmp.alloc_n<int64_t>(cnt_n);
        int64_t *off = tmp.alloc_n<int64_t>(cnt_n + 1);
        int64_t *base = tmp.alloc_n<int64_t>(1);
        set_i64(base, ne, s);
        const int nsides = h.same_xy ? 1 : 2;
        const int64_t nbnd = (int64_t)cnt_n * nsides * ((1 << g.bpl) - 1);
        int *bnd = tmp.alloc_n<int>(nbnd > 0 ? nbnd : 1);
        if (nbnd > 0) {
          k_tree_bounds<<<ceil_div(nbnd, 256), 256, 0, s>>>(N, nb, ne, kx, ky, lev - 1, h.leaf,
                                                            g, nsides, bnd);
          SMASH_CHECK_LAUNCH();
        }
        k_tree_split<<<ceil_div(cnt_n, 256), 256, 0, s>>>(N, nb, ne, lev - 1, h.leaf, g, nsides,
                                                          bnd, cnt, deeper);
        SMASH_CHECK_LAUNCH();
        scan_i64(cnt, off, cnt_n, base, s, tmp);
        const int64_t *pin = pick_words(s, {{off + cnt_n, 8}, {deeper, 4}});
        const int64_t total = pin[0] - ne;
        if (pin[1]) return true;
        if (total > 0) {
          if (ne + total > (int64_t)INT32_MAX) throw Error{SMASH_E_UNSUPPORTED, "too many nodes"};
          grow_nodes(h, cap, (int)(ne + total));
          refresh();
        }
        k_tree_emit<<<ceil_div(cnt_n, 256), 256, 0, s>>>(N, nb, ne, lev - 1, h.leaf, g, nsides,
                                                         bnd, off);
        SMASH_CHECK_LAUNCH();
        if (total == 0) return false;
        nb = ne;
        ne = (int)(ne + total);
        lev++;
      }
    };
    make_keys(x, h.nx, kx, px);
    if (!h.same_xy) make_keys(y, h.ny, ky, py);
    const int lead = std::min(g.max_split, std::max(1, 24 / g.bpl));
    bool full = lead == g.max_split || h.leaf > LS_MAX;
    g.split_cap = full ? g.max_split : lead;
    const int lo_bit = keybits - g.split_cap * g.bpl;
    sort_keys(kx, px, h.nx, lo_bit);
    if (!h.same_xy) sort_keys(ky, py, h.ny, lo_bit);
    if (h.same_xy) ky = kx;
    const bool deep = grow_tree();
    if (deep) {
      // a node needs deeper stages: sort the full keys and grow the tree again
      full = true;
      g.split_cap = g.max_split;
      make_keys(x, h.nx, kx, px);
      sort_keys(kx, px, h.nx, 0);
      if (!h.same_xy) {
        make_keys(y, h.ny, ky, py);
        sort_keys(ky, py, h.ny, 0);
      } else {
        ky = kx;
      }
      if (grow_tree()) throw Error{SMASH_E_DEVICE, "tree: full keys still too shallow"};
    }
    if (!full) {
      k_leaf_sort<<<ne, 64, 0, s>>>(h.nchild, h.xb, h.xe, ne, kx, px);
      SMASH_CHECK_LAUNCH();
      if (!h.same_xy) {
        k_leaf_sort<<<ne, 64, 0, s>>>(h.nchild, h.yb, h.ye, ne, ky, py);
        SMASH_CHECK_LAUNCH();
      }
    }
    h.perm_x = px;
    h.Xp = h.mem.alloc_n<double>((size_t)h.nx * h.d);
    k_gather_points<<<ceil_div(h.nx, 256), 256, 0, s>>>(x, px, h.nx, h.d, h.Xp);
    SMASH_CHECK_LAUNCH();
    if (h.pdata_in) {  // per-point data, permuted with the points
      h.Ap = h.mem.alloc_n<double>((size_t)h.nx * 3);
      k_gather_points<<<ceil_div(h.nx, 256), 256, 0, s>>>(h.pdata_in, px, h.nx, 3, h.Ap);
      SMASH_CHECK_LAUNCH();
    }
    if (h.same_xy) {
      h.perm_y = h.perm_x;
      h.Yp = h.Xp;
    } else {
      h.perm_y = py;
      h.Yp = h.mem.alloc_n<double>((size_t)h.ny * h.d);
      k_gather_points<<<ceil_div(h.ny, 256), 256, 0, s>>>(y, py, h.ny, h.d, h.Yp);
      SMASH_CHECK_LAUNCH();
    }
    h.nlevels = lev;
    h.nnodes = ne;
    defer_release(h, tmp);
  } catch (...) {
    (void)hipStreamSynchronize(s);
    tmp.release();
    throw;
  }
}

}  // namespace smash
