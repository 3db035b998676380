/*
 * smash_oracle.c -- plain, slow FP64 CPU reference for SMASH
 * (Cai, Chow, Saad, Xi, "SMASH: Structured Matrix Approximation by
 * Separation and Hierarchy", arXiv 1705.05443).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the
 * HIP library.
 *
 * Every step follows the paper in its own order and notation:
 *   kernel                      eq. (2.1) (and the three test kernels)
 *   adaptive partition          Sec. 3.1, Remark A.1
 *   well-separated test         Def. 2.1, eq. (2.3), on the boxes Omega_i
 *   admissible leaves L, L^-    eqs. (3.3), (3.4); HSS form eq. (3.5)
 *   near-field sets N_i         eq. (A.1)
 *   interpolation basis U-hat   eq. (2.2); Taylor basis eqs. (2.4)-(2.5)
 *   near-field truncated SVD    eqs. (3.7)-(3.8), (3.11)-(3.12), Def. 6.1
 *   compr (strong RRQR ID)      Thm. 2.4, eqs. (2.10)-(2.14)
 *   generators, parent grids    eqs. (3.6), (3.9)-(3.10), (3.13)-(3.14),
 *                               (3.16)-(3.18)
 *   coupling / near blocks      eqs. (3.15), (3.19), (3.20)
 *   matrix-vector product       Sec. 3.4, node-wise steps 1-3
 *   Cauchy-like product         eqs. (6.1), (6.2)
 *
 * Readings of points the paper leaves open are fixed here and listed with
 * the repository's design notes; each is named where it is used.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared.
 * Parallelism: OpenMP over the nodes of one tree level (the paper's own
 * level parallelism) and over row nodes in the product.  Every node's own
 * arithmetic is sequential, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_EUNSUP -2
#define OR_ENOMEM -3
#define OR_ENUMERIC -5

/* ------------------------------------------------------------------ */
/* Kernel functions.  Kernel 3 is eq. (2.1) restricted to the real line;
 * kernels 0-2 are the radial test kernels.  Kernel 4 is the Laplace
 * double layer of Sec. 6.4, eq. (6.9), in its Nystrom form: with
 * Phi(x, y) = -log|x - y| / (2 pi), the normal derivative at y times the
 * speed |r'| and the quadrature weight is grad_y Phi . m_y
 * = -((y - x) . m_y) / (2 pi |x - y|^2), where the column point's data
 * ay = (m_y1, m_y2, .) carries m_y = w (r2', -r1') (the outer normal of a
 * counterclockwise curve times |r'| w).  "x = y" means every coordinate
 * equal; then singular kernels return the chosen diagonal value d_x --
 * for kernel 4 the row point's own (ax[2]).                              */
/* ------------------------------------------------------------------ */
static double kernel_value(int kid, const double *x, const double *y, int d,
                           double diag, const double *ax, const double *ay) {
  int same = 1;
  double r2 = 0.0;
  for (int t = 0; t < d; t++) {
    double df = x[t] - y[t];
    if (x[t] != y[t]) same = 0;
    r2 += df * df;
  }
  if (kid == 2) return exp(-sqrt(r2));
  if (kid == 4) {
    if (same) return ax[2];
    double proj = (y[0] - x[0]) * ay[0] + (y[1] - x[1]) * ay[1];
    return -proj / (2.0 * M_PI * r2);
  }
  if (same) return diag;
  if (kid == 0) return 1.0 / sqrt(r2);
  if (kid == 1) return log(sqrt(r2));
  /* kid == 3: 1/(x - y) on the real line */
  return 1.0 / (x[0] - y[0]);
}

/* per-point data of point i (kernel 4), or NULL */
static const double *pd_at(const double *A, int64_t i) { return A ? A + 3 * i : NULL; }

/* ------------------------------------------------------------------ */
/* Adaptive partition (Sec. 3.1; Remark A.1 for the binary HSS tree).    */
/* ------------------------------------------------------------------ */
typedef struct {
  int d;          /* dimension                                  */
  int hss;        /* 1: binary tree, one axis per level         */
  int bpl;        /* key bits per split: d (2^d-tree) or 1      */
  int max_split;  /* number of bisection stages allowed         */
  double lo[3], hi[3];
} geom_t;

/* Full bisection key of one point: the sequence of half-box choices from
 * the root down through max_split stages, most significant first.  Point
 * x goes to the upper half of an axis iff x >= mid, mid = 0.5*(lo+hi).   */
static uint64_t point_key(const double *x, const geom_t *g) {
  double lo[3], hi[3];
  for (int t = 0; t < g->d; t++) {
    lo[t] = g->lo[t];
    hi[t] = g->hi[t];
  }
  uint64_t key = 0;
  for (int s = 0; s < g->max_split; s++) {
    for (int u = 0; u < g->bpl; u++) {
      int t = g->hss ? (s % g->d) : u;
      double mid = 0.5 * (lo[t] + hi[t]);
      int bit = x[t] >= mid;
      key = (key << 1) | (uint64_t)bit;
      if (bit)
        lo[t] = mid;
      else
        hi[t] = mid;
    }
  }
  return key;
}

typedef struct {
  uint64_t key;
  int idx;
} keyidx_t;

static int cmp_keyidx(const void *a, const void *b) {
  const keyidx_t *p = (const keyidx_t *)a, *q = (const keyidx_t *)b;
  if (p->key < q->key) return -1;
  if (p->key > q->key) return 1;
  return (p->idx > q->idx) - (p->idx < q->idx);
}

/* digit of split stage s (0-based) in a key with max_split stages */
static int key_digit(uint64_t key, int s, const geom_t *g) {
  int shift = (g->max_split - 1 - s) * g->bpl;
  return (int)((key >> shift) & ((1u << g->bpl) - 1u));
}

/* ------------------------------------------------------------------ */
/* Handle                                                              */
/* ------------------------------------------------------------------ */
typedef struct {
  int m, k;       /* grid size |i-bar| and rank |i-hat|                 */
  int *grid;      /* m permuted point ids, ascending                    */
  int *sel;       /* m local positions: k skeleton asc, then rest asc   */
  double *G;      /* (m-k) x k row-major                                */
  int ks;         /* HSS: number of kept singular vectors               */
  int nsw;        /* Gu-Eisenstat swaps performed                       */
  double gap;     /* smallest relative margin of a pivot choice         */
  double rgap;    /* relative margin of the rank cutoff (step k-1 kept,
                     step k dropped against tol * |R_11|)               */
  double sgap;    /* smallest relative margin of a swap decision: the
                     arg-max of rho against the runner-up, and the
                     winning rho against f                              */
  double vgap;    /* HSS: relative margin of the SVD truncation          */
} side_t;

typedef struct {
  int d, kid, adm, leaf, p, symmetric_reuse;
  double tol, tau, eps_svd, f, diag;
  double taylor_g; /* > 0: the Taylor basis of eqs. (2.4)-(2.5) (d = 1), g as there */
  int nx, ny;
  double *X, *Y;          /* permuted coordinates, n x d row-major */
  double *AX;             /* kernel 4: permuted per-point data, n x 3 (X = Y) */
  int *perm_x, *perm_y;   /* perm[a] = original index of permuted point a */
  geom_t g;
  /* nodes, BFS order (level by level, Morton order inside a level) */
  int nnodes, cap, nlevels;
  int *level, *parent, *first_child, *nchild, *xb, *xe, *yb, *ye;
  double *lo, *hi;        /* nnodes x 3 */
  int *level_beg;         /* nodes of level l (1-based): [level_beg[l-1], level_beg[l]) */
  /* admissible leaves L and inadmissible leaves L^- (sorted by (i,j)) */
  int nL, nLm;
  int *Li, *Lj, *Lmi, *Lmj;
  int *Lrow;              /* CSR row pointer of L by i (nnodes+1)  */
  int *Lmrow;             /* CSR row pointer of L^- by i           */
  /* HSS near-field sets N_i (CSR) */
  int *Nrow, *Ncol;
  side_t *row, *col;      /* per node; col == row when reused */
  int err;
} oracle_t;

static int is_leaf(const oracle_t *h, int i) { return h->nchild[i] == 0; }

static int grow_nodes(oracle_t *h) {
  int nc = h->cap ? 2 * h->cap : 64;
#define GROW(f, T)                                            \
  do {                                                        \
    T *p_ = (T *)realloc(h->f, sizeof(T) * (size_t)nc);       \
    if (!p_) return OR_ENOMEM;                                \
    h->f = p_;                                                \
  } while (0)
  GROW(level, int);
  GROW(parent, int);
  GROW(first_child, int);
  GROW(nchild, int);
  GROW(xb, int);
  GROW(xe, int);
  GROW(yb, int);
  GROW(ye, int);
#undef GROW
  double *l2 = (double *)realloc(h->lo, sizeof(double) * 3 * (size_t)nc);
  if (!l2) return OR_ENOMEM;
  h->lo = l2;
  double *h2 = (double *)realloc(h->hi, sizeof(double) * 3 * (size_t)nc);
  if (!h2) return OR_ENOMEM;
  h->hi = h2;
  h->cap = nc;
  return OR_OK;
}

/* Tree: keys, stable order, then nodes level by level.  A node is split iff
 * it holds more than nu_0 points of X or of Y and bisection stages remain;
 * empty boxes (no X and no Y point) are discarded (Sec. 3.1).            */
static int build_tree(oracle_t *h, const double *x, const double *y) {
  const geom_t *g = &h->g;
  int d = h->d;
  keyidx_t *kx = (keyidx_t *)malloc(sizeof(keyidx_t) * (size_t)(h->nx + 1));
  keyidx_t *ky = (keyidx_t *)malloc(sizeof(keyidx_t) * (size_t)(h->ny + 1));
  if (!kx || !ky) return OR_ENOMEM;
  for (int a = 0; a < h->nx; a++) {
    kx[a].key = point_key(x + (size_t)a * d, g);
    kx[a].idx = a;
  }
  for (int a = 0; a < h->ny; a++) {
    ky[a].key = point_key(y + (size_t)a * d, g);
    ky[a].idx = a;
  }
  qsort(kx, (size_t)h->nx, sizeof(keyidx_t), cmp_keyidx);
  qsort(ky, (size_t)h->ny, sizeof(keyidx_t), cmp_keyidx);
  h->perm_x = (int *)malloc(sizeof(int) * (size_t)(h->nx + 1));
  h->perm_y = (int *)malloc(sizeof(int) * (size_t)(h->ny + 1));
  h->X = (double *)malloc(sizeof(double) * (size_t)(h->nx * d + 1));
  h->Y = (double *)malloc(sizeof(double) * (size_t)(h->ny * d + 1));
  if (!h->perm_x || !h->perm_y || !h->X || !h->Y) return OR_ENOMEM;
  for (int a = 0; a < h->nx; a++) {
    h->perm_x[a] = kx[a].idx;
    for (int t = 0; t < d; t++) h->X[(size_t)a * d + t] = x[(size_t)kx[a].idx * d + t];
  }
  for (int a = 0; a < h->ny; a++) {
    h->perm_y[a] = ky[a].idx;
    for (int t = 0; t < d; t++) h->Y[(size_t)a * d + t] = y[(size_t)ky[a].idx * d + t];
  }

  if (grow_nodes(h)) return OR_ENOMEM;
  h->nnodes = 1;
  h->level[0] = 1;
  h->parent[0] = -1;
  h->xb[0] = 0;
  h->xe[0] = h->nx;
  h->yb[0] = 0;
  h->ye[0] = h->ny;
  for (int t = 0; t < 3; t++) {
    h->lo[t] = t < d ? g->lo[t] : 0.0;
    h->hi[t] = t < d ? g->hi[t] : 0.0;
  }
  int lvcap = 8;
  h->level_beg = (int *)malloc(sizeof(int) * (size_t)lvcap);
  h->level_beg[0] = 0;
  int beg = 0, end = 1, lev = 1;
  int nd = 1 << g->bpl;
  while (beg < end) {
    if (lev + 1 > lvcap - 1) {
      lvcap *= 2;
      h->level_beg = (int *)realloc(h->level_beg, sizeof(int) * (size_t)lvcap);
    }
    h->level_beg[lev] = end;
    for (int i = beg; i < end; i++) {
      int s = lev - 1; /* split stage that creates level lev+1 */
      int nxi = h->xe[i] - h->xb[i], nyi = h->ye[i] - h->yb[i];
      int split = (nxi > h->leaf || nyi > h->leaf) && s < g->max_split;
      h->first_child[i] = h->nnodes;
      h->nchild[i] = 0;
      if (!split) continue;
      int ax = h->xb[i], ay = h->yb[i];
      for (int v = 0; v < nd; v++) {
        int bx = ax, by = ay;
        while (bx < h->xe[i] && key_digit(kx[bx].key, s, g) == v) bx++;
        while (by < h->ye[i] && key_digit(ky[by].key, s, g) == v) by++;
        if (bx > ax || by > ay) {
          if (h->nnodes >= h->cap && grow_nodes(h)) return OR_ENOMEM;
          int c = h->nnodes++;
          h->level[c] = lev + 1;
          h->parent[c] = i;
          h->xb[c] = ax;
          h->xe[c] = bx;
          h->yb[c] = ay;
          h->ye[c] = by;
          h->first_child[c] = -1;
          h->nchild[c] = 0;
          for (int t = 0; t < 3; t++) {
            h->lo[3 * c + t] = h->lo[3 * i + t];
            h->hi[3 * c + t] = h->hi[3 * i + t];
          }
          /* child box: bisection of the parent box along the split axes */
          for (int u = 0; u < g->bpl; u++) {
            int t = g->hss ? (s % d) : u;
            int bit = (v >> (g->bpl - 1 - u)) & 1;
            double mid = 0.5 * (h->lo[3 * i + t] + h->hi[3 * i + t]);
            if (bit)
              h->lo[3 * c + t] = mid;
            else
              h->hi[3 * c + t] = mid;
          }
          h->nchild[i]++;
        }
        ax = bx;
        ay = by;
      }
    }
    beg = end;
    end = h->nnodes;
    lev++;
  }
  h->nlevels = lev - 1;
  h->level_beg[h->nlevels] = h->nnodes;
  free(kx);
  free(ky);
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Well-separated boxes, Def. 2.1 eq. (2.3): delta_i + delta_j <= tau|c_i-c_j|
 * with c the box center and delta half its diagonal, evaluated without a
 * square root:  e = tau^2 D^2 - delta_i^2 - delta_j^2 >= 0  and
 * 4 delta_i^2 delta_j^2 <= e^2.                                         */
/* ------------------------------------------------------------------ */
static int well_separated(const oracle_t *h, int i, int j) {
  double di2 = 0.0, dj2 = 0.0, D2 = 0.0;
  for (int t = 0; t < h->d; t++) {
    double wi = h->hi[3 * i + t] - h->lo[3 * i + t];
    double wj = h->hi[3 * j + t] - h->lo[3 * j + t];
    di2 += wi * wi;
    dj2 += wj * wj;
    double ci = 0.5 * (h->lo[3 * i + t] + h->hi[3 * i + t]);
    double cj = 0.5 * (h->lo[3 * j + t] + h->hi[3 * j + t]);
    double dc = ci - cj;
    D2 += dc * dc;
  }
  di2 = 0.25 * di2;
  dj2 = 0.25 * dj2;
  double e = h->tau * h->tau * D2 - di2 - dj2;
  if (e < 0.0) return 0;
  return 4.0 * di2 * dj2 <= e * e;
}

/* ------------------------------------------------------------------ */
/* Pair lists                                                          */
/* ------------------------------------------------------------------ */
typedef struct {
  int *i, *j;
  int n, cap;
} plist_t;

static int plist_push(plist_t *p, int i, int j) {
  if (p->n == p->cap) {
    int nc = p->cap ? 2 * p->cap : 256;
    int *a = (int *)realloc(p->i, sizeof(int) * (size_t)nc);
    if (!a) return OR_ENOMEM;
    p->i = a;
    int *b = (int *)realloc(p->j, sizeof(int) * (size_t)nc);
    if (!b) return OR_ENOMEM;
    p->j = b;
    p->cap = nc;
  }
  p->i[p->n] = i;
  p->j[p->n] = j;
  p->n++;
  return OR_OK;
}

static int cmp_pair(const void *a, const void *b) {
  const int *p = (const int *)a, *q = (const int *)b;
  if (p[0] != q[0]) return (p[0] > q[0]) - (p[0] < q[0]);
  return (p[1] > q[1]) - (p[1] < q[1]);
}

static int sort_pairs(plist_t *p, int **oi, int **oj) {
  int *buf = (int *)malloc(sizeof(int) * 2 * (size_t)(p->n + 1));
  if (!buf) return OR_ENOMEM;
  for (int a = 0; a < p->n; a++) {
    buf[2 * a] = p->i[a];
    buf[2 * a + 1] = p->j[a];
  }
  qsort(buf, (size_t)p->n, 2 * sizeof(int), cmp_pair);
  *oi = (int *)malloc(sizeof(int) * (size_t)(p->n + 1));
  *oj = (int *)malloc(sizeof(int) * (size_t)(p->n + 1));
  if (!*oi || !*oj) return OR_ENOMEM;
  for (int a = 0; a < p->n; a++) {
    (*oi)[a] = buf[2 * a];
    (*oj)[a] = buf[2 * a + 1];
  }
  free(buf);
  free(p->i);
  free(p->j);
  return OR_OK;
}

static int *csr_rows(const int *ii, int n, int nnodes) {
  int *r = (int *)calloc((size_t)nnodes + 1, sizeof(int));
  if (!r) return NULL;
  for (int a = 0; a < n; a++) r[ii[a] + 1]++;
  for (int i = 0; i < nnodes; i++) r[i + 1] += r[i];
  return r;
}

/* Strong admissibility, minimal admissible partition: eqs. (3.3), (3.4).
 * Dual traversal from (root, root): a separated pair of distinct nodes is
 * an admissible leaf; two leaves that are not separated form an
 * inadmissible leaf; otherwise both sides descend together while both are
 * inner nodes (they stay on one level), and only the inner side descends
 * once the other is a leaf.                                              */
static int h2_pairs(oracle_t *h) {
  plist_t L = {0}, Lm = {0}, st = {0};
  if (plist_push(&st, 0, 0)) return OR_ENOMEM;
  while (st.n > 0) {
    st.n--;
    int i = st.i[st.n], j = st.j[st.n];
    if (i != j && well_separated(h, i, j)) {
      if (plist_push(&L, i, j)) return OR_ENOMEM;
    } else if (is_leaf(h, i) && is_leaf(h, j)) {
      if (plist_push(&Lm, i, j)) return OR_ENOMEM;
    } else if (!is_leaf(h, i) && !is_leaf(h, j)) {
      for (int c = 0; c < h->nchild[i]; c++)
        for (int e = 0; e < h->nchild[j]; e++)
          if (plist_push(&st, h->first_child[i] + c, h->first_child[j] + e)) return OR_ENOMEM;
    } else if (is_leaf(h, i)) {
      for (int e = 0; e < h->nchild[j]; e++)
        if (plist_push(&st, i, h->first_child[j] + e)) return OR_ENOMEM;
    } else {
      for (int c = 0; c < h->nchild[i]; c++)
        if (plist_push(&st, h->first_child[i] + c, j)) return OR_ENOMEM;
    }
  }
  free(st.i);
  free(st.j);
  h->nL = L.n;
  h->nLm = Lm.n;
  if (sort_pairs(&L, &h->Li, &h->Lj)) return OR_ENOMEM;
  if (sort_pairs(&Lm, &h->Lmi, &h->Lmj)) return OR_ENOMEM;
  return OR_OK;
}

/* Weak admissibility (HSS), eq. (3.5): L = {(i, sibling of i)},
 * L^- = {(i, i) : i leaf}; and the near-field sets N_i of eq. (A.1),
 * built top-down: N_root is empty; N_i holds the siblings of i, the
 * children k of members of N_{p_i} with (i,k) not separated, and the
 * leaves k in N_{p_i} with (i,k) not separated.                         */
static int hss_pairs(oracle_t *h) {
  plist_t L = {0}, Lm = {0};
  for (int i = 1; i < h->nnodes; i++) {
    int p = h->parent[i];
    for (int c = 0; c < h->nchild[p]; c++) {
      int s = h->first_child[p] + c;
      if (s != i && plist_push(&L, i, s)) return OR_ENOMEM;
    }
  }
  for (int i = 0; i < h->nnodes; i++)
    if (is_leaf(h, i) && plist_push(&Lm, i, i)) return OR_ENOMEM;
  h->nL = L.n;
  h->nLm = Lm.n;
  if (sort_pairs(&L, &h->Li, &h->Lj)) return OR_ENOMEM;
  if (sort_pairs(&Lm, &h->Lmi, &h->Lmj)) return OR_ENOMEM;

  /* N_i, level by level (BFS order makes every parent precede its child) */
  int cap = 4 * h->nnodes + 16, n = 0;
  h->Nrow = (int *)calloc((size_t)h->nnodes + 1, sizeof(int));
  h->Ncol = (int *)malloc(sizeof(int) * (size_t)cap);
  if (!h->Nrow || !h->Ncol) return OR_ENOMEM;
  h->Nrow[0] = 0;
  h->Nrow[1] = 0; /* root: empty */
  for (int i = 1; i < h->nnodes; i++) {
    int p = h->parent[i];
    int need = h->nchild[p] + 8;
    for (int a = h->Nrow[p]; a < h->Nrow[p + 1]; a++) {
      int m = h->Ncol[a];
      need += is_leaf(h, m) ? 1 : h->nchild[m];
    }
    if (n + need > cap) {
      while (n + need > cap) cap *= 2;
      int *nc = (int *)realloc(h->Ncol, sizeof(int) * (size_t)cap);
      if (!nc) return OR_ENOMEM;
      h->Ncol = nc;
    }
    for (int c = 0; c < h->nchild[p]; c++) {
      int s = h->first_child[p] + c;
      if (s != i) h->Ncol[n++] = s;
    }
    for (int a = h->Nrow[p]; a < h->Nrow[p + 1]; a++) {
      int m = h->Ncol[a];
      if (is_leaf(h, m)) {
        if (!well_separated(h, i, m)) h->Ncol[n++] = m;
      } else {
        for (int c = 0; c < h->nchild[m]; c++) {
          int k = h->first_child[m] + c;
          if (!well_separated(h, i, k)) h->Ncol[n++] = k;
        }
      }
    }
    h->Nrow[i + 1] = n;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Far-field basis by interpolation, eq. (2.2): tensor Lagrange basis on p
 * first-kind Chebyshev points per axis mapped to the box Omega_i,
 * evaluated in barycentric form with weights (-1)^k sin((2k+1)pi/(2p)).
 * Column index k_1 p^{d-1} + ... + k_d.                                  */
/* ------------------------------------------------------------------ */
static void lagrange_1d(double x, double lo, double hi, int p, double *out) {
  if (hi - lo == 0.0) { /* degenerate box: constant basis */
    for (int k = 0; k < p; k++) out[k] = k == 0 ? 1.0 : 0.0;
    return;
  }
  double den = 0.0;
  for (int k = 0; k < p; k++) {
    double th = M_PI * (2.0 * k + 1.0) / (2.0 * p);
    double xi = 0.5 * (lo + hi) + 0.5 * (hi - lo) * cos(th);
    if (x == xi) {
      for (int j = 0; j < p; j++) out[j] = j == k ? 1.0 : 0.0;
      return;
    }
    double w = ((k & 1) ? -1.0 : 1.0) * sin(th);
    out[k] = w / (x - xi);
    den += out[k];
  }
  for (int k = 0; k < p; k++) out[k] = out[k] / den;
}

/* ------------------------------------------------------------------ */
/* Far-field basis by the Taylor expansion, eqs. (2.4)-(2.5), on the line:
 * the r = p functions phi_{a,l}(x - a) = eta_{a,l} (x - a)^l / l! of the box
 * [lo, hi], whose center a and radius delta (half its width) stand for
 * those of the set (Def. 2.1), with eta_{a,0} = 1 and
 * eta_{a,l} = (l g / delta)^l, g = (2 pi r)^{1/(2r)} / e, for l >= 1.  So
 * phi_l = (u l g)^l / l! with u = (x - a) / delta, taken as the running
 * product of (u l g) / k over k = 1..l.                                   */
/* ------------------------------------------------------------------ */
static double taylor_g_of(int r) { return pow(2.0 * M_PI * r, 1.0 / (2.0 * r)) / exp(1.0); }

static void taylor_1d(double x, double lo, double hi, int p, double g, double *out) {
  if (hi - lo == 0.0) { /* degenerate box: constant basis */
    for (int l = 0; l < p; l++) out[l] = l == 0 ? 1.0 : 0.0;
    return;
  }
  const double a = 0.5 * (lo + hi), del = 0.5 * (hi - lo);
  const double u = (x - a) / del;
  out[0] = 1.0;
  for (int l = 1; l < p; l++) {
    const double w = u * ((double)l * g);
    double v = 1.0;
    for (int k = 1; k <= l; k++) v = v * w / k;
    out[l] = v;
  }
}

/* C = U-hat (m x p^d) row-major for the m points pts (m x d) in the box:
 * the interpolation basis (2.2), or with g > 0 (d = 1) the Taylor basis. */
static void interp_basis(const double *pts, int m, int d, const double *lo,
                         const double *hi, int p, double g, double *C, int ldc) {
  double f[3][64];
  int c = 1;
  for (int t = 0; t < d; t++) c *= p;
  for (int a = 0; a < m; a++) {
    for (int t = 0; t < d; t++) {
      if (g > 0.0)
        taylor_1d(pts[(size_t)a * d + t], lo[t], hi[t], p, g, f[t]);
      else
        lagrange_1d(pts[(size_t)a * d + t], lo[t], hi[t], p, f[t]);
    }
    for (int col = 0; col < c; col++) {
      int r = col;
      double v = 1.0;
      for (int t = d - 1; t >= 0; t--) {
        v *= f[t][r % p];
        r /= p;
      }
      C[(size_t)a * ldc + col] = v;
    }
  }
}

/* ------------------------------------------------------------------ */
/* Truncated SVD for the HSS near-field block rows, eqs. (3.7)-(3.8).
 * One-sided (Hestenes) Jacobi on the rows of A (m x n): rotate pairs of
 * rows until all are mutually orthogonal; the accumulated rotations are
 * the left singular vectors, the row norms the singular values.  Keep the
 * vectors with sigma >= eps_svd * sigma_1 (Def. 6.1).  Writes S (m x ks,
 * row-major, columns by decreasing sigma) and returns ks.                */
/* ------------------------------------------------------------------ */
static int left_svd_truncated(double *A, int m, int n, double eps, double *S, int lds,
                              double *sig_out) {
  double *V = (double *)calloc((size_t)m * m + 1, sizeof(double));
  double *sg = (double *)malloc(sizeof(double) * (size_t)(m + 1));
  int *ord = (int *)malloc(sizeof(int) * (size_t)(m + 1));
  if (!V || !sg || !ord) return -1;
  for (int a = 0; a < m; a++) V[(size_t)a * m + a] = 1.0;
  for (int sweep = 0; sweep < 80; sweep++) {
    int rotated = 0;
    for (int pp = 0; pp < m - 1; pp++) {
      for (int qq = pp + 1; qq < m; qq++) {
        double *ap = A + (size_t)pp * n, *aq = A + (size_t)qq * n;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int t = 0; t < n; t++) {
          al += ap[t] * ap[t];
          be += aq[t] * aq[t];
          ga += ap[t] * aq[t];
        }
        if (al == 0.0 || be == 0.0) continue;
        if (fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
        rotated = 1;
        double zeta = (be - al) / (2.0 * ga);
        double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double cs = 1.0 / sqrt(1.0 + tt * tt);
        double sn = cs * tt;
        for (int t = 0; t < n; t++) {
          double u = ap[t], v = aq[t];
          ap[t] = cs * u - sn * v;
          aq[t] = sn * u + cs * v;
        }
        /* columns pp, qq of V accumulate the same rotation */
        for (int t = 0; t < m; t++) {
          double u = V[(size_t)t * m + pp], v = V[(size_t)t * m + qq];
          V[(size_t)t * m + pp] = cs * u - sn * v;
          V[(size_t)t * m + qq] = sn * u + cs * v;
        }
      }
    }
    if (!rotated) break;
  }
  for (int a = 0; a < m; a++) {
    double s = 0.0;
    for (int t = 0; t < n; t++) s += A[(size_t)a * n + t] * A[(size_t)a * n + t];
    sg[a] = sqrt(s);
    ord[a] = a;
  }
  /* order by decreasing sigma, ties by index (insertion sort: m is small) */
  for (int a = 1; a < m; a++) {
    int v = ord[a], b = a - 1;
    while (b >= 0 && (sg[ord[b]] < sg[v])) {
      ord[b + 1] = ord[b];
      b--;
    }
    ord[b + 1] = v;
  }
  int ks = 0;
  double s1 = m > 0 ? sg[ord[0]] : 0.0;
  if (s1 > 0.0)
    for (int a = 0; a < m; a++)
      if (sg[ord[a]] >= eps * s1) ks = a + 1;
  for (int c = 0; c < ks; c++)
    for (int t = 0; t < m; t++) S[(size_t)t * lds + c] = V[(size_t)t * m + ord[c]];
  if (sig_out)
    for (int a = 0; a < m; a++) sig_out[a] = sg[ord[a]];
  free(V);
  free(sg);
  free(ord);
  return ks;
}

/* ------------------------------------------------------------------ */
/* compr(C, i-bar), eq. (2.14): strong rank-revealing QR (Thm. 2.4) applied
 * to M = C^T (c x m), written as an interpolative decomposition
 * C = P [I; G] C|_{i-hat}, eq. (2.11).
 *   (i)   Householder QR with column pivoting on M; the pivot is the column
 *         of largest residual 2-norm, recomputed from the transformed
 *         columns at every step; ties go to the lowest position.
 *   (ii)  rank k = number of steps with residual norm > tol * |R_11|.
 *   (iii) Gu-Eisenstat swaps: with N = R11^{-1} R12, 1/omega_i the norm of
 *         row i of R11^{-1} and gamma_j the norm of column j of R22, swap
 *         the pair maximising rho_ij = sqrt(N_ij^2 + (gamma_j/omega_i)^2)
 *         while it exceeds f (ties: smallest j, then smallest i), and
 *         refactor without pivoting.
 *   (iv)  G = N^T with skeleton and remaining rows both in ascending order.
 * C is m x c row-major.  Output: *k, sel[m] (k skeleton positions
 * ascending, then the m-k others ascending), G ((m-k) x k row-major).   */
/* ------------------------------------------------------------------ */
static void householder_step(double *W, int c, int m, int t) {
  /* W column-major: column a at W + a*c; reflect column t onto e_t */
  double *x = W + (size_t)t * c;
  double s2 = 0.0;
  for (int r = t; r < c; r++) s2 += x[r] * x[r];
  double alpha = sqrt(s2);
  if (alpha == 0.0) return;
  double rtt = x[t] >= 0.0 ? -alpha : alpha;
  double *v = (double *)malloc(sizeof(double) * (size_t)(c - t));
  v[0] = x[t] - rtt;
  for (int r = t + 1; r < c; r++) v[r - t] = x[r];
  double vn = 0.0;
  for (int r = 0; r < c - t; r++) vn += v[r] * v[r];
  if (vn > 0.0) {
    for (int a = t + 1; a < m; a++) {
      double *y = W + (size_t)a * c;
      double w = 0.0;
      for (int r = t; r < c; r++) w += v[r - t] * y[r];
      double sc = 2.0 * w / vn;
      for (int r = t; r < c; r++) y[r] -= sc * v[r - t];
    }
  }
  x[t] = rtt;
  for (int r = t + 1; r < c; r++) x[r] = 0.0;
  free(v);
}

/* margins (test diagnostics only, NULL to skip): [0] smallest relative gap
 * between the chosen pivot norm and the runner-up; [1] relative distance of
 * the norms at the rank cutoff from tol * |R_11|; [2] smallest relative gap
 * of a swap decision (winning rho against the runner-up and against f).   */
static int compr(const double *C, int m, int c, double tol, double f, int *k_out, int *sel,
                 double *G, int *nswaps, double *margins) {
  *nswaps = 0;
  double *min_gap = margins;
  if (margins) margins[0] = margins[1] = margins[2] = 1.0;
  if (m == 0) {
    *k_out = 0;
    return OR_OK;
  }
  double *W = (double *)malloc(sizeof(double) * (size_t)m * c);
  int *perm = (int *)malloc(sizeof(int) * (size_t)m);
  if (!W || !perm) return OR_ENOMEM;
  for (int a = 0; a < m; a++) {
    perm[a] = a;
    memcpy(W + (size_t)a * c, C + (size_t)a * c, sizeof(double) * (size_t)c);
  }
  int kmax = m < c ? m : c;
  int k = 0;
  double r00 = 0.0;
  for (int t = 0; t < kmax; t++) {
    int best = -1;
    double bn = -1.0, b2 = -1.0; /* largest and second largest residual norm */
    for (int a = t; a < m; a++) {
      double s = 0.0;
      const double *y = W + (size_t)a * c;
      for (int r = t; r < c; r++) s += y[r] * y[r];
      double nr = sqrt(s);
      if (nr > bn) {
        b2 = bn;
        bn = nr;
        best = a;
      } else if (nr > b2) {
        b2 = nr;
      }
    }
    if (t == 0) {
      r00 = bn;
      if (r00 == 0.0) break;
    } else {
      double cut = tol * r00;
      if (margins && cut > 0.0 && fabs(bn - cut) / cut < margins[1]) margins[1] = fabs(bn - cut) / cut;
      if (bn <= cut) break;
    }
    /* relative margin of this pivot choice (a test diagnostic only) */
    if (min_gap && b2 >= 0.0 && (bn - b2) / bn < *min_gap) *min_gap = (bn - b2) / bn;
    if (best != t) {
      for (int r = 0; r < c; r++) {
        double tmp = W[(size_t)t * c + r];
        W[(size_t)t * c + r] = W[(size_t)best * c + r];
        W[(size_t)best * c + r] = tmp;
      }
      int tp = perm[t];
      perm[t] = perm[best];
      perm[best] = tp;
    }
    householder_step(W, c, m, t);
    k = t + 1;
  }

  int nr = m - k;
  double *N = NULL, *Ri = NULL, *gam = NULL, *rinv = NULL;
  if (k > 0 && nr > 0) {
    N = (double *)malloc(sizeof(double) * (size_t)k * nr);
    Ri = (double *)malloc(sizeof(double) * (size_t)k * k);
    gam = (double *)malloc(sizeof(double) * (size_t)nr);
    rinv = (double *)malloc(sizeof(double) * (size_t)k);
    if (!N || !Ri || !gam || !rinv) return OR_ENOMEM;
    for (;;) {
      /* N = R11^{-1} R12 by back substitution; R(r, a) = W[a*c + r] */
      for (int j = 0; j < nr; j++) {
        const double *y = W + (size_t)(k + j) * c;
        for (int i = k - 1; i >= 0; i--) {
          double s = y[i];
          for (int q = i + 1; q < k; q++) s -= W[(size_t)q * c + i] * N[(size_t)q * nr + j];
          N[(size_t)i * nr + j] = s / W[(size_t)i * c + i];
        }
        double g2 = 0.0;
        for (int r = k; r < c; r++) g2 += y[r] * y[r];
        gam[j] = sqrt(g2);
      }
      /* R11^{-1}, column by column (upper triangular) */
      for (int j = 0; j < k; j++) {
        for (int i = k - 1; i >= 0; i--) {
          double s = (i == j) ? 1.0 : 0.0;
          for (int q = i + 1; q < k; q++) s -= W[(size_t)q * c + i] * Ri[(size_t)q * k + j];
          Ri[(size_t)i * k + j] = s / W[(size_t)i * c + i];
        }
      }
      for (int i = 0; i < k; i++) {
        double s = 0.0;
        for (int j = 0; j < k; j++) s += Ri[(size_t)i * k + j] * Ri[(size_t)i * k + j];
        rinv[i] = sqrt(s); /* = 1/omega_i */
      }
      double best = -1.0, second = -1.0;
      int bi = -1, bj = -1;
      for (int j = 0; j < nr; j++) {
        for (int i = 0; i < k; i++) {
          double a = N[(size_t)i * nr + j];
          double b = gam[j] * rinv[i];
          double rho = sqrt(a * a + b * b);
          if (rho > best) {
            second = best;
            best = rho;
            bi = i;
            bj = j;
          } else if (rho > second) {
            second = rho;
          }
        }
      }
      if (margins) {
        double gf = fabs(best - f) / f;
        if (gf < margins[2]) margins[2] = gf;
        if (best > f && second >= 0.0 && (best - second) / best < margins[2])
          margins[2] = (best - second) / best;
      }
      if (!(best > f)) break;
      if (++(*nswaps) > 64 * k) {
        free(W);
        free(perm);
        free(N);
        free(Ri);
        free(gam);
        free(rinv);
        return OR_ENUMERIC;
      }
      /* swap skeleton position bi with remaining position k+bj, refactor */
      int tp = perm[bi];
      perm[bi] = perm[k + bj];
      perm[k + bj] = tp;
      for (int a = 0; a < m; a++) memcpy(W + (size_t)a * c, C + (size_t)perm[a] * c, sizeof(double) * (size_t)c);
      for (int t = 0; t < k; t++) householder_step(W, c, m, t);
    }
  }
  /* canonical order: skeleton ascending, remaining ascending */
  int *sk = (int *)malloc(sizeof(int) * (size_t)(k + 1));
  int *rs = (int *)malloc(sizeof(int) * (size_t)(nr + 1));
  int *pos_sk = (int *)malloc(sizeof(int) * (size_t)(m + 1));
  int *pos_rs = (int *)malloc(sizeof(int) * (size_t)(m + 1));
  char *is_sk = (char *)calloc((size_t)m + 1, 1);
  for (int i = 0; i < k; i++) is_sk[perm[i]] = 1;
  int a1 = 0, a2 = 0;
  for (int a = 0; a < m; a++) {
    if (is_sk[a]) {
      pos_sk[a] = a1;
      sk[a1++] = a;
    } else {
      pos_rs[a] = a2;
      rs[a2++] = a;
    }
  }
  for (int i = 0; i < k; i++) sel[i] = sk[i];
  for (int j = 0; j < nr; j++) sel[k + j] = rs[j];
  if (k > 0 && nr > 0) {
    for (int i = 0; i < k; i++)
      for (int j = 0; j < nr; j++) {
        int row = pos_rs[perm[k + j]], col = pos_sk[perm[i]];
        G[(size_t)row * k + col] = N[(size_t)i * nr + j];
      }
  }
  *k_out = k;
  free(sk);
  free(rs);
  free(pos_sk);
  free(pos_rs);
  free(is_sk);
  free(W);
  free(perm);
  free(N);
  free(Ri);
  free(gam);
  free(rinv);
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Level-wise construction, Sec. 3.3.                                 */
/* ------------------------------------------------------------------ */
static int ipow(int b, int e) {
  int r = 1;
  while (e-- > 0) r *= b;
  return r;
}

/* current grid of node i on one side (eqs. (3.6), (3.14), (3.18)):
 * a leaf's own points; otherwise the children's skeletons in child order */
static int side_grid(oracle_t *h, side_t *sd, int i, int rowside) {
  side_t *s = &sd[i];
  if (is_leaf(h, i)) {
    int b = rowside ? h->xb[i] : h->yb[i], e = rowside ? h->xe[i] : h->ye[i];
    s->m = e - b;
    s->grid = (int *)malloc(sizeof(int) * (size_t)(s->m + 1));
    if (!s->grid) return OR_ENOMEM;
    for (int a = 0; a < s->m; a++) s->grid[a] = b + a;
  } else {
    int m = 0;
    for (int c = 0; c < h->nchild[i]; c++) m += sd[h->first_child[i] + c].k;
    s->m = m;
    s->grid = (int *)malloc(sizeof(int) * (size_t)(m + 1));
    if (!s->grid) return OR_ENOMEM;
    int o = 0;
    for (int c = 0; c < h->nchild[i]; c++) {
      side_t *cs = &sd[h->first_child[i] + c];
      for (int t = 0; t < cs->k; t++) s->grid[o++] = cs->grid[cs->sel[t]];
    }
  }
  return OR_OK;
}

/* HSS near-field block row (3.7) of node i on one side; returns a malloc'd
 * m x n matrix and its column count.  For the row side the columns are the
 * column grids of N_i (concatenated in N_i order); for the column side
 * (3.11) the roles of X and Y swap.                                        */
static double *near_block(oracle_t *h, int i, int rowside, int *ncols) {
  side_t *me = rowside ? h->row : h->col;
  side_t *ot = rowside ? h->col : h->row;
  int n = 0;
  for (int a = h->Nrow[i]; a < h->Nrow[i + 1]; a++) n += ot[h->Ncol[a]].m;
  *ncols = n;
  int m = me[i].m;
  double *A = (double *)malloc(sizeof(double) * ((size_t)m * n + 1));
  if (!A) return NULL;
  int o = 0;
  for (int a = h->Nrow[i]; a < h->Nrow[i + 1]; a++) {
    side_t *js = &ot[h->Ncol[a]];
    for (int b = 0; b < js->m; b++) {
      for (int r = 0; r < m; r++) {
        const int xi = rowside ? me[i].grid[r] : js->grid[b];
        const int yi = rowside ? js->grid[b] : me[i].grid[r];
        A[(size_t)r * n + o] =
            kernel_value(h->kid, h->X + (size_t)xi * h->d, h->Y + (size_t)yi * h->d, h->d,
                         h->diag, pd_at(h->AX, xi), pd_at(h->AX, yi));
      }
      o++;
    }
  }
  return A;
}

static int compress_node(oracle_t *h, int i, int rowside) {
  side_t *s = rowside ? &h->row[i] : &h->col[i];
  int d = h->d, pd = ipow(h->p, d);
  /* kernel 4, column side: kappa(x, y) = m_y . grad_y Phi(x, y), a sum of
   * two functions of y smooth away from x, each weighted by a component of
   * m_y: the basis is [m_y1 U-hat(y), m_y2 U-hat(y)] (width 2 p^d)       */
  const int dl_col = h->kid == 4 && !rowside;
  int c0 = dl_col ? 2 * pd : pd;
  int m = s->m;
  const double *P = rowside ? h->X : h->Y;
  double *S = NULL;
  int ks = 0;
  s->gap = s->rgap = s->sgap = s->vgap = 1.0;
  if (h->adm == 0 && m > 0) {
    int nc = 0;
    double *A = near_block(h, i, rowside, &nc);
    if (!A) return OR_ENOMEM;
    if (nc > 0) {
      S = (double *)malloc(sizeof(double) * ((size_t)m * m + 1));
      double *sig = (double *)malloc(sizeof(double) * ((size_t)m + 1));
      if (!S || !sig) return OR_ENOMEM;
      ks = left_svd_truncated(A, m, nc, h->eps_svd, S, m, sig);
      if (ks < 0) return OR_ENOMEM;
      /* diagnostic: how close any singular value lies to the cutoff */
      double cut = h->eps_svd * sig[0];
      for (int a = 0; a < m && cut > 0.0; a++)
        if (fabs(sig[a] - cut) / cut < s->vgap) s->vgap = fabs(sig[a] - cut) / cut;
      free(sig);
    }
    free(A);
  }
  s->ks = ks;
  int c = c0 + ks;
  s->sel = (int *)malloc(sizeof(int) * (size_t)(m + 1));
  if (!s->sel) return OR_ENOMEM;
  if (m == 0) {
    s->k = 0;
    s->G = NULL;
    free(S);
    return OR_OK;
  }
  double *C = (double *)malloc(sizeof(double) * (size_t)m * c);
  double *pts = (double *)malloc(sizeof(double) * (size_t)m * d);
  if (!C || !pts) return OR_ENOMEM;
  for (int a = 0; a < m; a++)
    for (int t = 0; t < d; t++) pts[(size_t)a * d + t] = P[(size_t)s->grid[a] * d + t];
  double lo[3], hi[3];
  for (int t = 0; t < d; t++) {
    lo[t] = h->lo[3 * i + t];
    hi[t] = h->hi[3 * i + t];
  }
  interp_basis(pts, m, d, lo, hi, h->p, h->taylor_g, C, c);
  if (dl_col)
    for (int a = 0; a < m; a++) {
      const double *da = h->AX + (size_t)s->grid[a] * 3;
      double *Ca = C + (size_t)a * c;
      for (int q = 0; q < pd; q++) {
        Ca[pd + q] = da[1] * Ca[q];
        Ca[q] = da[0] * Ca[q];
      }
    }
  for (int a = 0; a < m; a++)
    for (int q = 0; q < ks; q++) C[(size_t)a * c + c0 + q] = S[(size_t)a * m + q];
  s->G = (double *)malloc(sizeof(double) * ((size_t)m * c + 1));
  if (!s->G) return OR_ENOMEM;
  int nsw = 0;
  double mg[3];
  int rc = compr(C, m, c, h->tol, h->f, &s->k, s->sel, s->G, &nsw, mg);
  s->gap = mg[0];
  s->rgap = mg[1];
  s->sgap = mg[2];
  s->nsw = nsw;
  free(C);
  free(pts);
  free(S);
  return rc;
}

static int build_generators(oracle_t *h) {
  h->row = (side_t *)calloc((size_t)h->nnodes, sizeof(side_t));
  if (!h->row) return OR_ENOMEM;
  if (h->symmetric_reuse)
    h->col = h->row;
  else {
    h->col = (side_t *)calloc((size_t)h->nnodes, sizeof(side_t));
    if (!h->col) return OR_ENOMEM;
  }
  int err = OR_OK;
  /* leaf grids are the leaves' own points (3.6); they are needed before
   * their own level is reached, as near-field columns of finer nodes */
  for (int i = 1; i < h->nnodes; i++) {
    if (!is_leaf(h, i)) continue;
    if (side_grid(h, h->row, i, 1)) return OR_ENOMEM;
    if (!h->symmetric_reuse && side_grid(h, h->col, i, 0)) return OR_ENOMEM;
  }
  for (int l = h->nlevels; l >= 2; l--) {
    int b = h->level_beg[l - 1], e = h->level_beg[l];
    /* inner-node grids of this level, from the level below (3.14), (3.18) */
    for (int i = b; i < e; i++) {
      if (is_leaf(h, i)) continue;
      if (side_grid(h, h->row, i, 1)) return OR_ENOMEM;
      if (!h->symmetric_reuse && side_grid(h, h->col, i, 0)) return OR_ENOMEM;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = b; i < e; i++) {
      int rc = compress_node(h, i, 1);
      if (rc == OR_OK && !h->symmetric_reuse) rc = compress_node(h, i, 0);
      if (rc != OR_OK) {
#pragma omp critical
        err = rc;
      }
    }
    if (err) return err;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Public entry points                                                */
/* ------------------------------------------------------------------ */
static void free_side(side_t *s, int n) {
  if (!s) return;
  for (int i = 0; i < n; i++) {
    free(s[i].grid);
    free(s[i].sel);
    free(s[i].G);
  }
  free(s);
}

void oracle_destroy(void *hv) {
  oracle_t *h = (oracle_t *)hv;
  if (!h) return;
  if (h->col != h->row) free_side(h->col, h->nnodes);
  free_side(h->row, h->nnodes);
  free(h->X);
  free(h->Y);
  free(h->AX);
  free(h->perm_x);
  free(h->perm_y);
  free(h->level);
  free(h->parent);
  free(h->first_child);
  free(h->nchild);
  free(h->xb);
  free(h->xe);
  free(h->yb);
  free(h->ye);
  free(h->lo);
  free(h->hi);
  free(h->level_beg);
  free(h->Li);
  free(h->Lj);
  free(h->Lmi);
  free(h->Lmj);
  free(h->Lrow);
  free(h->Lmrow);
  free(h->Nrow);
  free(h->Ncol);
  free(h);
}

/* x: nx x d, y: ny x d (row-major, original order).  same_xy != 0 means Y
 * is X (then the column side is reused for symmetric kernels).  adm: 0 weak
 * (HSS, binary tree), 1 strong (H^2, 2^d-tree).  root: if has_root, the box
 * [root_lo, root_lo + root_side]^d, else the bounding cube of X and Y.     */
/* data: kernel 4 only, the per-point data of the points (n x 3, original
 * order: m_1, m_2, diagonal value); X = Y is required for kernel 4.      */
static int build_impl(const double *x, int64_t nx, const double *y, int64_t ny, int same_xy,
                      int d, int kid, int leaf, int p, int adm, double tol, double tau,
                      double eps_svd, double f, double diag, int has_root, const double *root_lo,
                      double root_side, int max_depth, const double *data, int tree_only,
                      int basis, void **out);

int oracle_build(const double *x, int64_t nx, const double *y, int64_t ny, int same_xy,
                 int d, int kid, int leaf, int p, int adm, double tol, double tau,
                 double eps_svd, double f, double diag, int has_root, const double *root_lo,
                 double root_side, int max_depth, const double *data, void **out) {
  return build_impl(x, nx, y, ny, same_xy, d, kid, leaf, p, adm, tol, tau, eps_svd, f, diag,
                    has_root, root_lo, root_side, max_depth, data, 0, 0, out);
}

/* The same with a choice of far-field basis: 0 the interpolation basis
 * (2.2), 1 the Taylor basis (2.4)-(2.5) with r = p terms (d = 1 only). */
int oracle_build_basis(const double *x, int64_t nx, const double *y, int64_t ny, int same_xy,
                       int d, int kid, int leaf, int p, int adm, double tol, double tau,
                       double eps_svd, double f, double diag, int has_root,
                       const double *root_lo, double root_side, int max_depth,
                       const double *data, int basis, void **out) {
  return build_impl(x, nx, y, ny, same_xy, d, kid, leaf, p, adm, tol, tau, eps_svd, f, diag,
                    has_root, root_lo, root_side, max_depth, data, 0, basis, out);
}

/* The partition and the pair lists only (Sec. 3.1, eqs. (3.3)-(3.5), (A.1)):
 * for tests that need the tree of a large case without its generators.
 * Exports that need generators return OR_EUNSUP.                          */
int oracle_build_tree(const double *x, int64_t nx, const double *y, int64_t ny, int same_xy,
                      int d, int kid, int leaf, int adm, double tau, int has_root,
                      const double *root_lo, double root_side, int max_depth, const double *data,
                      void **out) {
  return build_impl(x, nx, y, ny, same_xy, d, kid, leaf, 1, adm, 0.0, tau, 0.0, 2.0, 0.0,
                    has_root, root_lo, root_side, max_depth, data, 1, 0, out);
}

static int build_impl(const double *x, int64_t nx, const double *y, int64_t ny, int same_xy,
                      int d, int kid, int leaf, int p, int adm, double tol, double tau,
                      double eps_svd, double f, double diag, int has_root, const double *root_lo,
                      double root_side, int max_depth, const double *data, int tree_only,
                      int basis, void **out) {
  *out = NULL;
  if (d < 1 || d > 3 || nx < 1 || ny < 1 || leaf < 1 || p < 1 || p > 64 || tau <= 0.0 ||
      tau >= 1.0 || f <= 1.0 || tol < 0.0 || (adm != 0 && adm != 1) || kid < 0 || kid > 4)
    return OR_EINVAL;
  if (kid == 3 && d != 1) return OR_EUNSUP;
  if (kid == 4 && (d != 2 || !same_xy || !data)) return OR_EUNSUP;
  if (basis != 0 && (basis != 1 || d != 1 || kid == 4)) return OR_EUNSUP;
  if (kid == 4)
    for (int64_t a = 0; a < nx * 3; a++)
      if (!isfinite(data[a])) return OR_ENUMERIC;
  oracle_t *h = (oracle_t *)calloc(1, sizeof(oracle_t));
  if (!h) return OR_ENOMEM;
  h->d = d;
  h->kid = kid;
  h->adm = adm;
  h->leaf = leaf;
  h->p = p;
  h->taylor_g = basis == 1 ? taylor_g_of(p) : 0.0;
  h->tol = tol;
  h->tau = tau;
  h->eps_svd = eps_svd;
  h->f = f;
  h->diag = diag;
  h->nx = (int)nx;
  h->ny = (int)ny;
  h->symmetric_reuse = same_xy && kid != 3 && kid != 4;
  h->g.d = d;
  h->g.hss = adm == 0;
  h->g.bpl = adm == 0 ? 1 : d;
  h->g.max_split = 63 / h->g.bpl;
  if (max_depth > 0 && max_depth - 1 < h->g.max_split) h->g.max_split = max_depth - 1;
  for (int64_t a = 0; a < nx * d; a++)
    if (!isfinite(x[a])) {
      free(h);
      return OR_ENUMERIC;
    }
  for (int64_t a = 0; a < ny * d; a++)
    if (!isfinite(y[a])) {
      free(h);
      return OR_ENUMERIC;
    }
  if (has_root) {
    for (int t = 0; t < d; t++) {
      h->g.lo[t] = root_lo[t];
      h->g.hi[t] = root_lo[t] + root_side;
    }
    for (int64_t a = 0; a < nx; a++)
      for (int t = 0; t < d; t++)
        if (!(x[a * d + t] >= h->g.lo[t] && x[a * d + t] <= h->g.hi[t])) {
          free(h);
          return OR_EINVAL;
        }
    for (int64_t a = 0; a < ny; a++)
      for (int t = 0; t < d; t++)
        if (!(y[a * d + t] >= h->g.lo[t] && y[a * d + t] <= h->g.hi[t])) {
          free(h);
          return OR_EINVAL;
        }
  } else {
    /* bounding cube of X and Y */
    double side = 0.0;
    for (int t = 0; t < d; t++) {
      double mn = x[t], mx = x[t];
      for (int64_t a = 0; a < nx; a++) {
        double v = x[a * d + t];
        if (v < mn) mn = v;
        if (v > mx) mx = v;
      }
      for (int64_t a = 0; a < ny; a++) {
        double v = y[a * d + t];
        if (v < mn) mn = v;
        if (v > mx) mx = v;
      }
      h->g.lo[t] = mn;
      if (mx - mn > side) side = mx - mn;
    }
    for (int t = 0; t < d; t++) h->g.hi[t] = h->g.lo[t] + side;
  }
  int rc = build_tree(h, x, y);
  if (!rc && kid == 4) {
    h->AX = (double *)malloc(sizeof(double) * (size_t)h->nx * 3);
    if (!h->AX) rc = OR_ENOMEM;
    for (int a = 0; !rc && a < h->nx; a++)
      for (int c = 0; c < 3; c++) h->AX[(size_t)a * 3 + c] = data[(size_t)h->perm_x[a] * 3 + c];
  }
  if (!rc) rc = adm == 1 ? h2_pairs(h) : hss_pairs(h);
  if (!rc) {
    h->Lrow = csr_rows(h->Li, h->nL, h->nnodes);
    h->Lmrow = csr_rows(h->Lmi, h->nLm, h->nnodes);
    if (!h->Lrow || !h->Lmrow) rc = OR_ENOMEM;
  }
  if (!rc && !tree_only) rc = build_generators(h);
  if (rc) {
    oracle_destroy(h);
    return rc;
  }
  *out = h;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Matrix-vector product, Sec. 3.4, node-wise form (steps 1-3), applied to
 * every leaf at whatever level it sits; coupling and near-field blocks are
 * evaluated from the kernel on the fly, eqs. (3.19), (3.20).
 * Q: ny x R, Z: nx x R, both row-major in the ORIGINAL point order.      */
/* ------------------------------------------------------------------ */
static void apply_id_t(const side_t *s, const double *g, int R, double *out) {
  /* out (k x R) = g|_hat + G^T g|_check,  g: m x R */
  int k = s->k, nr = s->m - s->k;
  for (int t = 0; t < k; t++)
    for (int r = 0; r < R; r++) out[(size_t)t * R + r] = g[(size_t)s->sel[t] * R + r];
  for (int a = 0; a < nr; a++) {
    const double *ga = g + (size_t)s->sel[k + a] * R;
    for (int t = 0; t < k; t++) {
      double w = s->G[(size_t)a * k + t];
      for (int r = 0; r < R; r++) out[(size_t)t * R + r] += w * ga[r];
    }
  }
}

static void apply_id(const side_t *s, const double *zh, int R, double *zbar) {
  /* zbar (m x R) += P [I; G] zh,  zh: k x R */
  int k = s->k, nr = s->m - s->k;
  for (int t = 0; t < k; t++)
    for (int r = 0; r < R; r++) zbar[(size_t)s->sel[t] * R + r] += zh[(size_t)t * R + r];
  for (int a = 0; a < nr; a++) {
    double *za = zbar + (size_t)s->sel[k + a] * R;
    for (int t = 0; t < k; t++) {
      double w = s->G[(size_t)a * k + t];
      for (int r = 0; r < R; r++) za[r] += w * zh[(size_t)t * R + r];
    }
  }
}

int oracle_matvec(void *hv, const double *Q, int64_t R64, double *Z) {
  oracle_t *h = (oracle_t *)hv;
  if (!h->row) return OR_EUNSUP; /* a tree-only build */
  int R = (int)R64;
  int d = h->d;
  double *q = (double *)malloc(sizeof(double) * ((size_t)h->ny * R + 1));
  double *z = (double *)calloc((size_t)h->nx * R + 1, sizeof(double));
  double **qh = (double **)calloc((size_t)h->nnodes, sizeof(double *));
  double **zh = (double **)calloc((size_t)h->nnodes, sizeof(double *));
  if (!q || !z || !qh || !zh) return OR_ENOMEM;
  for (int a = 0; a < h->ny; a++)
    for (int r = 0; r < R; r++) q[(size_t)a * R + r] = Q[(size_t)h->perm_y[a] * R + r];
  for (int i = 1; i < h->nnodes; i++) {
    qh[i] = (double *)calloc((size_t)h->col[i].k * R + 1, sizeof(double));
    zh[i] = (double *)calloc((size_t)h->row[i].k * R + 1, sizeof(double));
    if (!qh[i] || !zh[i]) return OR_ENOMEM;
  }
  /* step 1: upward pass, q-hat_i = V_i^T q|_i or sum_c W_c^T q-hat_c */
  for (int l = h->nlevels; l >= 2; l--) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = h->level_beg[l - 1]; i < h->level_beg[l]; i++) {
      const side_t *s = &h->col[i];
      double *g = (double *)malloc(sizeof(double) * ((size_t)s->m * R + 1));
      if (is_leaf(h, i)) {
        memcpy(g, q + (size_t)h->yb[i] * R, sizeof(double) * (size_t)s->m * R);
      } else {
        int o = 0;
        for (int c = 0; c < h->nchild[i]; c++) {
          int ch = h->first_child[i] + c;
          memcpy(g + (size_t)o * R, qh[ch], sizeof(double) * (size_t)h->col[ch].k * R);
          o += h->col[ch].k;
        }
      }
      apply_id_t(s, g, R, qh[i]);
      free(g);
    }
  }
  /* step 2: z-hat_i = sum over (i,j) in L of B_ij q-hat_j, B_ij = A|(i-hat, j-hat) */
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 1; i < h->nnodes; i++) {
    const side_t *si = &h->row[i];
    for (int a = h->Lrow[i]; a < h->Lrow[i + 1]; a++) {
      int j = h->Lj[a];
      const side_t *sj = &h->col[j];
      for (int t = 0; t < si->k; t++) {
        const int xi = si->grid[si->sel[t]];
        const double *xp = h->X + (size_t)xi * d;
        for (int u = 0; u < sj->k; u++) {
          const int yi = sj->grid[sj->sel[u]];
          const double *yp = h->Y + (size_t)yi * d;
          double b = kernel_value(h->kid, xp, yp, d, h->diag, pd_at(h->AX, xi), pd_at(h->AX, yi));
          for (int r = 0; r < R; r++) zh[i][(size_t)t * R + r] += b * qh[j][(size_t)u * R + r];
        }
      }
    }
  }
  /* step 3: downward pass; leaves add U_i z-hat_i to z|_i */
  for (int l = 2; l <= h->nlevels; l++) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = h->level_beg[l - 1]; i < h->level_beg[l]; i++) {
      const side_t *s = &h->row[i];
      if (is_leaf(h, i)) {
        apply_id(s, zh[i], R, z + (size_t)h->xb[i] * R);
      } else {
        double *zb = (double *)calloc((size_t)s->m * R + 1, sizeof(double));
        apply_id(s, zh[i], R, zb);
        int o = 0;
        for (int c = 0; c < h->nchild[i]; c++) {
          int ch = h->first_child[i] + c;
          for (int t = 0; t < h->row[ch].k * R; t++) zh[ch][t] += zb[(size_t)o * R + t];
          o += h->row[ch].k;
        }
        free(zb);
      }
    }
  }
  /* near field: z|_i += sum over (i,j) in L^- of A|(i, j) q|_j */
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 0; i < h->nnodes; i++) {
    for (int a = h->Lmrow[i]; a < h->Lmrow[i + 1]; a++) {
      int j = h->Lmj[a];
      for (int u = h->xb[i]; u < h->xe[i]; u++) {
        const double *xp = h->X + (size_t)u * d;
        for (int v = h->yb[j]; v < h->ye[j]; v++) {
          double b = kernel_value(h->kid, xp, h->Y + (size_t)v * d, d, h->diag, pd_at(h->AX, u),
                                  pd_at(h->AX, v));
          for (int r = 0; r < R; r++) z[(size_t)u * R + r] += b * q[(size_t)v * R + r];
        }
      }
    }
  }
  for (int a = 0; a < h->nx; a++)
    for (int r = 0; r < R; r++) Z[(size_t)h->perm_x[a] * R + r] = z[(size_t)a * R + r];
  for (int i = 1; i < h->nnodes; i++) {
    free(qh[i]);
    free(zh[i]);
  }
  free(qh);
  free(zh);
  free(q);
  free(z);
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Export of the construction for comparisons.  With buf == NULL only the
 * element count is returned.                                          */
/* ------------------------------------------------------------------ */
enum {
  EX_PERM_X = 1, EX_PERM_Y = 2, EX_NODES = 3, EX_BOXES = 4, EX_L = 5, EX_LM = 6,
  EX_NEAR_PTR = 7, EX_NEAR_IDX = 8, EX_RANKS = 9, EX_ROW_SEL = 10, EX_ROW_G = 11,
  EX_COL_SEL = 12, EX_COL_G = 13, EX_ROW_GRID = 14, EX_COL_GRID = 15, EX_SIZES = 16,
  EX_LEVELS = 17, EX_SWAPS = 18, EX_MARGINS = 19, EX_DECISION_MARGINS = 20
};

int oracle_export(void *hv, int what, void *buf, int64_t *count) {
  oracle_t *h = (oracle_t *)hv;
  int64_t n = 0;
  int *ib = (int *)buf;
  double *db = (double *)buf;
  int nn = h->nnodes;
  if (!h->row && what >= EX_RANKS && what != EX_SIZES && what != EX_LEVELS)
    return OR_EUNSUP; /* generators of a tree-only build */
  switch (what) {
    case EX_SIZES: /* int32: nx, ny, nnodes, nlevels, nL, nLm, d, adm */
      n = 8;
      if (buf) {
        ib[0] = h->nx; ib[1] = h->ny; ib[2] = nn; ib[3] = h->nlevels;
        ib[4] = h->nL; ib[5] = h->nLm; ib[6] = h->d; ib[7] = h->adm;
      }
      break;
    case EX_LEVELS:
      n = h->nlevels + 1;
      if (buf) memcpy(ib, h->level_beg, sizeof(int) * (size_t)n);
      break;
    case EX_PERM_X:
      n = h->nx;
      if (buf) memcpy(ib, h->perm_x, sizeof(int) * (size_t)n);
      break;
    case EX_PERM_Y:
      n = h->ny;
      if (buf) memcpy(ib, h->perm_y, sizeof(int) * (size_t)n);
      break;
    case EX_NODES: /* int32 x 8: level, parent, first_child, nchild, xb, xe, yb, ye */
      n = (int64_t)nn * 8;
      if (buf)
        for (int i = 0; i < nn; i++) {
          int *o = ib + (size_t)i * 8;
          o[0] = h->level[i]; o[1] = h->parent[i];
          o[2] = h->nchild[i] ? h->first_child[i] : -1; o[3] = h->nchild[i];
          o[4] = h->xb[i]; o[5] = h->xe[i]; o[6] = h->yb[i]; o[7] = h->ye[i];
        }
      break;
    case EX_BOXES: /* double x 6: lo[3], hi[3] */
      n = (int64_t)nn * 6;
      if (buf)
        for (int i = 0; i < nn; i++)
          for (int t = 0; t < 3; t++) {
            db[(size_t)i * 6 + t] = h->lo[3 * i + t];
            db[(size_t)i * 6 + 3 + t] = h->hi[3 * i + t];
          }
      break;
    case EX_L:
      n = (int64_t)h->nL * 2;
      if (buf)
        for (int a = 0; a < h->nL; a++) { ib[2 * a] = h->Li[a]; ib[2 * a + 1] = h->Lj[a]; }
      break;
    case EX_LM:
      n = (int64_t)h->nLm * 2;
      if (buf)
        for (int a = 0; a < h->nLm; a++) { ib[2 * a] = h->Lmi[a]; ib[2 * a + 1] = h->Lmj[a]; }
      break;
    case EX_NEAR_PTR:
      n = h->Nrow ? nn + 1 : 0;
      if (buf && n) memcpy(ib, h->Nrow, sizeof(int) * (size_t)n);
      break;
    case EX_NEAR_IDX:
      n = h->Nrow ? h->Nrow[nn] : 0;
      if (buf && n) memcpy(ib, h->Ncol, sizeof(int) * (size_t)n);
      break;
    case EX_RANKS: /* int32 x 6: m_row, k_row, m_col, k_col, ks_row, ks_col (root: zeros) */
      n = (int64_t)nn * 6;
      if (buf)
        for (int i = 0; i < nn; i++) {
          int *o = ib + (size_t)i * 6;
          o[0] = h->row[i].m; o[1] = h->row[i].k; o[2] = h->col[i].m; o[3] = h->col[i].k;
          o[4] = h->row[i].ks; o[5] = h->col[i].ks;
        }
      break;
    case EX_MARGINS: /* double x 2: smallest relative pivot margin, row and column side */
      n = (int64_t)nn * 2;
      if (buf)
        for (int i = 0; i < nn; i++) {
          db[2 * i] = h->row[i].gap;
          db[2 * i + 1] = h->col[i].gap;
        }
      break;
    case EX_DECISION_MARGINS: /* double x 8 per node: pivot, rank cutoff, swap,
                                 SVD cutoff margins of the row side, then the
                                 column side (1.0: no such decision) */
      n = (int64_t)nn * 8;
      if (buf)
        for (int i = 0; i < nn; i++) {
          const side_t *sd[2] = {&h->row[i], &h->col[i]};
          for (int u = 0; u < 2; u++) {
            double *o = db + (size_t)i * 8 + 4 * u;
            int done = sd[u]->sel != NULL;
            o[0] = done ? sd[u]->gap : 1.0;
            o[1] = done ? sd[u]->rgap : 1.0;
            o[2] = done ? sd[u]->sgap : 1.0;
            o[3] = (done && h->adm == 0) ? sd[u]->vgap : 1.0;
          }
        }
      break;
    case EX_SWAPS: /* int32 x 2: swaps of the row and column side per node */
      n = (int64_t)nn * 2;
      if (buf)
        for (int i = 0; i < nn; i++) {
          ib[2 * i] = h->row[i].nsw;
          ib[2 * i + 1] = h->col[i].nsw;
        }
      break;
    case EX_ROW_SEL:
    case EX_COL_SEL:
    case EX_ROW_GRID:
    case EX_COL_GRID: {
      side_t *sd = (what == EX_ROW_SEL || what == EX_ROW_GRID) ? h->row : h->col;
      int grid = what == EX_ROW_GRID || what == EX_COL_GRID;
      for (int i = 1; i < nn; i++) {
        if (buf) memcpy(ib + n, grid ? sd[i].grid : sd[i].sel, sizeof(int) * (size_t)sd[i].m);
        n += sd[i].m;
      }
      break;
    }
    case EX_ROW_G:
    case EX_COL_G: {
      side_t *sd = what == EX_ROW_G ? h->row : h->col;
      for (int i = 1; i < nn; i++) {
        int64_t c = (int64_t)(sd[i].m - sd[i].k) * sd[i].k;
        if (buf && c) memcpy(db + n, sd[i].G, sizeof(double) * (size_t)c);
        n += c;
      }
      break;
    }
    default:
      return OR_EINVAL;
  }
  *count = n;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Exact references and single-step entry points for the pins.        */
/* ------------------------------------------------------------------ */
/* Z = A Q with A = [kappa(x, y)] (x in X, y in Y), original order. */
/* ax, ay: per-point data (n x 3, kernel 4) of X and Y, else NULL.      */
void oracle_dense_matvec(const double *x, int64_t nx, const double *y, int64_t ny, int d,
                         int kid, double diag, const double *ax, const double *ay,
                         const double *Q, int64_t R, double *Z) {
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < nx; a++) {
    double *za = Z + a * R;
    for (int64_t r = 0; r < R; r++) za[r] = 0.0;
    for (int64_t b = 0; b < ny; b++) {
      double v = kernel_value(kid, x + a * d, y + b * d, d, diag, pd_at(ax, a), pd_at(ay, b));
      for (int64_t r = 0; r < R; r++) za[r] += v * Q[b * R + r];
    }
  }
}

/* Cauchy-like matrix with generators w (nx x p) and v (ny x p), row-major,
 * eq. (6.1): a_ij = kappa(x_i, y_j) * sum_l w_il v_jl with the 1/(x - y)
 * kernel (kid 3, d = 1) on the real line; Z = A Q (original order). */
void oracle_cauchy_like_dense(const double *x, int64_t nx, const double *y, int64_t ny,
                              const double *w, const double *v, int p, const double *Q,
                              int64_t R, double *Z) {
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < nx; a++) {
    double *za = Z + a * R;
    for (int64_t r = 0; r < R; r++) za[r] = 0.0;
    for (int64_t b = 0; b < ny; b++) {
      double g = 0.0;
      for (int l = 0; l < p; l++) g += w[a * p + l] * v[b * p + l];
      const double e = kernel_value(3, x + a, y + b, 1, 0.0, NULL, NULL) * g;
      for (int64_t r = 0; r < R; r++) za[r] += e * Q[b * R + r];
    }
  }
}

/* The same product through the SMASH approximation C-hat of the Cauchy
 * matrix held by hv, by eq. (6.2): A = sum_l diag(w_l) C diag(v_l), so
 * Z = sum_l w_l o (C-hat (v_l o Q)), the terms added for l = 0, 1, ... */
int oracle_cauchy_like_matvec(void *hv, const double *w, const double *v, int p,
                              const double *Q, int64_t R, double *Z) {
  oracle_t *h = (oracle_t *)hv;
  double *ql = (double *)malloc(sizeof(double) * ((size_t)h->ny * R + 1));
  double *zl = (double *)malloc(sizeof(double) * ((size_t)h->nx * R + 1));
  if (!ql || !zl) {
    free(ql);
    free(zl);
    return OR_ENOMEM;
  }
  for (int64_t a = 0; a < (int64_t)h->nx * R; a++) Z[a] = 0.0;
  int rc = 0;
  for (int l = 0; l < p && rc == 0; l++) {
    for (int64_t b = 0; b < h->ny; b++)
      for (int64_t r = 0; r < R; r++) ql[b * R + r] = v[b * p + l] * Q[b * R + r];
    rc = oracle_matvec(hv, ql, R, zl);
    if (rc != 0) break;
    for (int64_t a = 0; a < h->nx; a++)
      for (int64_t r = 0; r < R; r++) Z[a * R + r] = Z[a * R + r] + w[a * p + l] * zl[a * R + r];
  }
  free(ql);
  free(zl);
  return rc;
}

/* rows[0..nrows) of A Q (exact), for sampled checks at large n. */
void oracle_dense_rows(const double *x, int64_t nx, const double *y, int64_t ny, int d,
                       int kid, double diag, const double *ax, const double *ay,
                       const int64_t *rows, int64_t nrows, const double *Q, int64_t R,
                       double *Z) {
  (void)nx;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < nrows; s++) {
    const double *xa = x + rows[s] * d;
    double *za = Z + s * R;
    for (int64_t r = 0; r < R; r++) za[r] = 0.0;
    for (int64_t b = 0; b < ny; b++) {
      double v = kernel_value(kid, xa, y + b * d, d, diag, pd_at(ax, rows[s]), pd_at(ay, b));
      for (int64_t r = 0; r < R; r++) za[r] += v * Q[b * R + r];
    }
  }
}

/* kernel block K(P[ri], Q[cj]) for given row/column points (n x d each). */
void oracle_kernel_block(const double *P, const double *Qp, int64_t nr, int64_t nc, int d,
                         int kid, double diag, const double *aP, const double *aQ, double *B) {
  for (int64_t a = 0; a < nr; a++)
    for (int64_t b = 0; b < nc; b++)
      B[a * nc + b] = kernel_value(kid, P + a * d, Qp + b * d, d, diag, pd_at(aP, a),
                                   pd_at(aQ, b));
}

int oracle_compr(const double *C, int m, int c, double tol, double f, int *k, int *sel,
                 double *G, int *nswaps) {
  return compr(C, m, c, tol, f, k, sel, G, nswaps, NULL);
}

void oracle_interp_basis(const double *pts, int m, int d, const double *lo, const double *hi,
                         int p, double *C) {
  interp_basis(pts, m, d, lo, hi, p, 0.0, C, ipow(p, d));
}

/* The Taylor basis (2.4)-(2.5) of the interval [lo, hi] with r = p terms at
 * m points (m x p row-major), for the pins. */
void oracle_taylor_basis(const double *pts, int m, double lo, double hi, int p, double *C) {
  interp_basis(pts, m, 1, &lo, &hi, p, taylor_g_of(p), C, p);
}

int oracle_left_svd(const double *A, int m, int n, double eps, double *S, double *sig) {
  double *W = (double *)malloc(sizeof(double) * ((size_t)m * n + 1));
  if (!W) return -1;
  memcpy(W, A, sizeof(double) * (size_t)m * n);
  int ks = left_svd_truncated(W, m, n, eps, S, m, sig);
  free(W);
  return ks;
}

int oracle_well_separated_boxes(const double *lo_i, const double *hi_i, const double *lo_j,
                                const double *hi_j, int d, double tau) {
  oracle_t h;
  double lo[6] = {0}, hi[6] = {0};
  memset(&h, 0, sizeof(h));
  for (int t = 0; t < d; t++) {
    lo[t] = lo_i[t];
    hi[t] = hi_i[t];
    lo[3 + t] = lo_j[t];
    hi[3 + t] = hi_j[t];
  }
  h.d = d;
  h.tau = tau;
  h.lo = lo;
  h.hi = hi;
  return well_separated(&h, 0, 1);
}

uint64_t oracle_point_key(const double *x, int d, int adm, const double *lo, const double *hi,
                          int max_split) {
  geom_t g;
  memset(&g, 0, sizeof(g));
  g.d = d;
  g.hss = adm == 0;
  g.bpl = adm == 0 ? 1 : d;
  g.max_split = max_split;
  for (int t = 0; t < d; t++) {
    g.lo[t] = lo[t];
    g.hi[t] = hi[t];
  }
  return point_key(x, &g);
}

/* Sec. 6.1 parameter heuristic: expansion order r for a target tolerance eps
 * once the separation ratio tau is chosen (three tolerance bands). */
int oracle_order_rule(double eps, double tau) {
  double q = log(eps) / log(tau);
  if (eps < 1e-8) return (int)floor(q - 20.0);
  if (eps < 1e-6) return (int)floor(q - 15.0);
  int r = (int)floor(q - 10.0);
  return r > 5 ? r : 5;
}
