// matvec.hip -- the product z = A-hat q of Sec. 3.4 (node-wise steps 1-3,
// batched one tree level per launch, eqs. (3.24)-(3.26) in level form):
//   gather    q = Q[perm_y]                        (slot region 0)
//   up        q-hat_i = q|_hat + H_i^T q|_check     levels L..2, column side
//   coupling  z-hat_i = sum_{(i,j) in L} B_ij q-hat_j   all nodes at once
//   down      z-bar|_hat += z-hat_i, z-bar|_check += G_i z-hat_i  levels 2..L
//             (a leaf writes its own points; an inner node adds into its
//             children's z-hat)
//   near+out  Z[perm_x] = z + sum_{(i,j) in L^-} B_ij q|_j
// Vectors live in the slot space of each side, nrhs values per slot
// (row-major), so a node's grid is a contiguous block of rows.
#include "common.cuh"

namespace smash {

constexpr int MV_NT = 256;

template <class T>
__global__ void __launch_bounds__(MV_NT) k_mv_gather(const T *__restrict__ X, int64_t ldx,
                                                     const int *__restrict__ perm, int64_t n,
                                                     int R, T *__restrict__ q) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  int64_t a = e / R;
  int r = (int)(e - a * R);
  q[e] = X[(int64_t)perm[a] * ldx + r];
}

struct SweepArgs {
  int nb, ne;
  const int *m, *k, *nchild;
  const int64_t *gbeg, *hbeg, *selo, *go;
  const int *sel;
  const void *G;
};

// q-hat_i[t] = g[sel[t]] + sum_a H[a][t] g[sel[k+a]]   (g = grid rows)
template <class T>
__global__ void __launch_bounds__(MV_NT) k_mv_up(SweepArgs A, T *__restrict__ q, int R) {
  const int i = A.nb + blockIdx.x;
  if (i >= A.ne) return;
  const int m = A.m[i], k = A.k[i];
  if (k == 0) return;
  const T *g = q + A.gbeg[i] * R;
  T *out = q + A.hbeg[i] * R;
  const int *sel = A.sel + A.selo[i];
  const T *H = (const T *)A.G + A.go[i];
  const int nr = m - k;
  for (int e = threadIdx.x; e < k * R; e += MV_NT) {
    const int t = e / R, r = e - t * R;
    T acc = g[(int64_t)sel[t] * R + r];
    for (int a = 0; a < nr; a++) acc += H[(int64_t)a * k + t] * g[(int64_t)sel[k + a] * R + r];
    out[(int64_t)t * R + r] = acc;
  }
}

// z-hat_i = sum over the L row of i of B_ij q-hat_j  (B column-major)
struct CouplingArgs {
  int nnodes;
  const int *Lrow, *Lj;
  const int64_t *boff;
  const int *krow, *kcol;
  const int64_t *hrow, *hcol;
  const void *B;
};

template <class T>
__global__ void __launch_bounds__(MV_NT) k_mv_coupling(CouplingArgs A, const T *__restrict__ qh,
                                                       T *__restrict__ zh, int R) {
  const int i = 1 + blockIdx.x;
  if (i >= A.nnodes) return;
  const int ki = A.krow[i];
  if (ki == 0) return;
  T *out = zh + A.hrow[i] * R;
  const T *Bv = (const T *)A.B;
  for (int e = threadIdx.x; e < ki * R; e += MV_NT) {
    const int t = e / R, r = e - t * R;
    T acc = 0;
    for (int p = A.Lrow[i]; p < A.Lrow[i + 1]; p++) {
      const int j = A.Lj[p];
      const int kj = A.kcol[j];
      const T *Bp = Bv + A.boff[p] + t;
      const T *qj = qh + A.hcol[j] * R + r;
      for (int s = 0; s < kj; s++) acc += Bp[(int64_t)s * ki] * qj[(int64_t)s * R];
    }
    out[(int64_t)t * R + r] = acc;
  }
}

// grid rows += P [I; G] z-hat_i (a leaf assigns: its rows are written once)
template <class T>
__global__ void __launch_bounds__(MV_NT) k_mv_down(SweepArgs A, T *__restrict__ z, int R) {
  const int i = A.nb + blockIdx.x;
  if (i >= A.ne) return;
  const int m = A.m[i], k = A.k[i];
  if (m == 0) return;
  const bool leaf = A.nchild[i] == 0;
  T *g = z + A.gbeg[i] * R;
  const T *zh = z + A.hbeg[i] * R;
  const int *sel = A.sel + A.selo[i];
  const T *G = (const T *)A.G + A.go[i];
  for (int e = threadIdx.x; e < m * R; e += MV_NT) {
    const int a = e / R, r = e - a * R;
    T v;
    if (a < k) {
      v = zh[(int64_t)a * R + r];
    } else {
      const T *Ga = G + (int64_t)(a - k) * k;
      v = 0;
      for (int t = 0; t < k; t++) v += Ga[t] * zh[(int64_t)t * R + r];
    }
    T *dst = g + (int64_t)sel[a] * R + r;
    if (leaf)
      *dst = v;
    else
      *dst += v;
  }
}

struct NearArgs {
  int nnodes;
  const int *nchild, *xb, *xe, *yb, *ye, *perm_x;
  const int *Lmrow, *Lmj;
  const int64_t *nboff;
  const void *Bn;
  int has_far;
};

template <class T>
__global__ void __launch_bounds__(MV_NT) k_mv_near_out(NearArgs A, const T *__restrict__ q,
                                                       const T *__restrict__ z, T *__restrict__ Y,
                                                       int64_t ldy, int R) {
  const int i = blockIdx.x;
  if (i >= A.nnodes || A.nchild[i] != 0) return;
  const int xb = A.xb[i], ni = A.xe[i] - xb;
  const T *Bv = (const T *)A.Bn;
  for (int e = threadIdx.x; e < ni * R; e += MV_NT) {
    const int a = e / R, r = e - a * R;
    T acc = A.has_far ? z[(int64_t)(xb + a) * R + r] : (T)0;
    for (int p = A.Lmrow[i]; p < A.Lmrow[i + 1]; p++) {
      const int j = A.Lmj[p];
      const int yb = A.yb[j], nj = A.ye[j] - yb;
      const T *Bp = Bv + A.nboff[p] + a;
      const T *qj = q + (int64_t)yb * R + r;
      for (int b = 0; b < nj; b++) acc += Bp[(int64_t)b * ni] * qj[(int64_t)b * R];
    }
    Y[(int64_t)A.perm_x[xb + a] * ldy + r] = acc;
  }
}

template <class T>
static void matvec_t(Handle &h, const T *X, int64_t ldx, int nrhs, T *Y, int64_t ldy,
                     hipStream_t s) {
  const int RC = 64;  // right-hand sides per pass
  Side &Rw = h.row, &Cl = *h.col;
  int chunk = nrhs < RC ? nrhs : RC;
  if (h.ws_nrhs != chunk) {
    h.ws_mem.stream = s;
    h.ws_mem.release();
    h.qbuf = h.ws_mem.alloc(sizeof(T) * (size_t)Cl.nslots * chunk);
    h.zbuf = h.ws_mem.alloc(sizeof(T) * (size_t)Rw.nslots * chunk);
    h.ws_nrhs = chunk;
  }
  T *q = (T *)h.qbuf, *z = (T *)h.zbuf;
  const bool f64 = h.apply_prec == SMASH_F64;
  for (int c0 = 0; c0 < nrhs; c0 += chunk) {
    const int R = nrhs - c0 < chunk ? nrhs - c0 : chunk;
    {
      PhaseTimer pt(h, SMASH_PHASE_MV_GATHER, s);
      k_mv_gather<T><<<ceil_div(h.ny * R, MV_NT), MV_NT, 0, s>>>(X + c0, ldx, h.perm_y, h.ny, R,
                                                                  q);
      SMASH_CHECK_LAUNCH();
    }
    const bool has_far = h.nlevels >= 2;
    {
    PhaseTimer pt(h, SMASH_PHASE_MV_UP, s);
    for (int l = h.nlevels; l >= 2; l--) {
      int nb = h.level_beg[l - 1], ne = h.level_beg[l];
      const LevelSide &L = Cl.lv[l];
      SweepArgs sa{nb, ne, Cl.m, Cl.k, h.nchild, Cl.gbeg, Cl.hbeg, Cl.selo, Cl.go, L.sel,
                   f64 ? (const void *)L.G : (const void *)L.G32};
      if (h.batched) {
        k_mv_up<T><<<ne - nb, MV_NT, 0, s>>>(sa, q, R);
        SMASH_CHECK_LAUNCH();
      } else {
        for (int i = nb; i < ne; i++) {
          sa.nb = i;
          sa.ne = i + 1;
          k_mv_up<T><<<1, MV_NT, 0, s>>>(sa, q, R);
          SMASH_CHECK_LAUNCH();
        }
      }
    }
    }
    if (has_far) {
      CouplingArgs ca{h.nnodes, h.Lrow, h.Lj, h.boff, Rw.k, Cl.k, Rw.hbeg, Cl.hbeg, h.B};
      {
        PhaseTimer pt(h, SMASH_PHASE_MV_COUPLING, s);
        k_mv_coupling<T><<<h.nnodes - 1, MV_NT, 0, s>>>(ca, q, z, R);
        SMASH_CHECK_LAUNCH();
      }
      PhaseTimer pt(h, SMASH_PHASE_MV_DOWN, s);
      for (int l = 2; l <= h.nlevels; l++) {
        int nb = h.level_beg[l - 1], ne = h.level_beg[l];
        const LevelSide &L = Rw.lv[l];
        SweepArgs sa{nb, ne, Rw.m, Rw.k, h.nchild, Rw.gbeg, Rw.hbeg, Rw.selo, Rw.go, L.sel,
                     f64 ? (const void *)L.G : (const void *)L.G32};
        if (h.batched) {
          k_mv_down<T><<<ne - nb, MV_NT, 0, s>>>(sa, z, R);
          SMASH_CHECK_LAUNCH();
        } else {
          for (int i = nb; i < ne; i++) {
            sa.nb = i;
            sa.ne = i + 1;
            k_mv_down<T><<<1, MV_NT, 0, s>>>(sa, z, R);
            SMASH_CHECK_LAUNCH();
          }
        }
      }
    }
    NearArgs na{h.nnodes, h.nchild, h.xb, h.xe, h.yb, h.ye, h.perm_x, h.Lmrow, h.Lmj, h.nboff,
                h.Bn, has_far ? 1 : 0};
    {
      PhaseTimer pt(h, SMASH_PHASE_MV_NEAR_OUT, s);
      k_mv_near_out<T><<<h.nnodes, MV_NT, 0, s>>>(na, q, z, Y + c0, ldy, R);
      SMASH_CHECK_LAUNCH();
    }
  }
}

void run_matvec(Handle &h, const void *X, int64_t ldx, int nrhs, void *Y, int64_t ldy,
                hipStream_t s) {
  if (h.apply_prec == SMASH_F64)
    matvec_t<double>(h, (const double *)X, ldx, nrhs, (double *)Y, ldy, s);
  else
    matvec_t<float>(h, (const float *)X, ldx, nrhs, (float *)Y, ldy, s);
}

}  // namespace smash
