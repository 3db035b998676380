// matvec.hip -- the product z = A-hat q of Sec. 3.4 (node-wise steps 1-3,
// batched one tree level per launch, eqs. (3.24)-(3.26) in level form):
//   gather    q = Q[perm_y]                        (slot region 0)
//   up        q-hat_i = q|_hat + H_i^T q|_check     levels L..2, column side
//   coupling  z-hat_i = sum_{(i,j) in L} B_ij q-hat_j   all nodes at once
//   down      z-bar|_hat += z-hat_i, z-bar|_check += G_i z-hat_i  levels 2..L
//             (a leaf writes its own points; an inner node adds into its
//             children's z-hat)
//   near+out  Z[perm_x] = z + sum_{(i,j) in L^-} B_ij q|_j
// Vectors live in the slot space of each side with RP values per slot
// (row-major; RP = the right-hand-side count rounded up to 16, padding
// columns hold zeros), so a node's grid is a contiguous block of rows.
//
// Every dense piece is a small matrix product C (rows x 16) += A (rows x K)
// * Bv (K x 16) with A one of G^T, G, B_ij and Bv a set of vector rows.  The
// sweeps run one to four wavefronts per node and 16-column tile; the
// coupling and near products one workgroup per node whose waves each cover
// every column tile, so each block is read once.  All use 16x16x4 MFMA: lane l feeds A[row0 + l%16][k0 + l/16] and
// Bv[k0 + l/16][col0 + l%16] and holds four results C[row][col0 + l%16]:
// row = row0 + 4(l/16) + e for the FP32 instruction and row0 + 4e + l/16
// for the FP64 one (e = 0..3; measured on gfx950).  A is stored with
// consecutive rows consecutive in memory, so each wave load is four
// 128-byte segments.
#include <mutex>

#include "common.cuh"

namespace smash {

constexpr int MV_NT = 64;
constexpr int MV_TILES = 4;  // 16-row tiles per pass (64 rows)

template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output row (within the 16-row tile) of result e held by lane group lk
  static __device__ __forceinline__ int row(int lk, int e) { return 4 * e + lk; }
};
template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int e) { return 4 * lk + e; }
};

template <class T>
__global__ void __launch_bounds__(256) k_mv_gather(const T *__restrict__ X, int64_t ldx,
                                                   const int *__restrict__ perm, int64_t n, int R,
                                                   int RP, T *__restrict__ q) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * RP) return;
  int64_t a = e / RP;
  int r = (int)(e - a * RP);
  q[e] = r < R ? X[(int64_t)perm[a] * ldx + r] : (T)0;
}

struct SweepArgs {
  int nb, ne;
  const int *m, *k, *nchild;
  const int64_t *gbeg, *hbeg, *selo, *go;
  const int *sel;
  const void *G;   // (m-k) x k row-major: as A = H^T it is column-major k x (m-k)
  const void *Gt;  // k x (m-k) row-major: as A = G it is column-major (m-k) x k
};

// Sum of the W partial accumulator tiles of a workgroup into wave 0 (LDS,
// one slot per wave, tile, result and lane).
template <class T, int W>
__device__ __forceinline__ void reduce_waves(typename Mfma<T>::acc_t (&acc)[MV_TILES], T *red) {
  const int w = threadIdx.x / MV_NT, l = threadIdx.x & (MV_NT - 1);
  __syncthreads();
  if (w > 0)
#pragma unroll
    for (int tt = 0; tt < MV_TILES; tt++)
#pragma unroll
      for (int e = 0; e < 4; e++) red[(((w - 1) * MV_TILES + tt) * 4 + e) * MV_NT + l] = acc[tt][e];
  __syncthreads();
  if (w == 0)
#pragma unroll
    for (int tt = 0; tt < MV_TILES; tt++)
#pragma unroll
      for (int e = 0; e < 4; e++)
        for (int v = 0; v < W - 1; v++) acc[tt][e] += red[((v * MV_TILES + tt) * 4 + e) * MV_NT + l];
}

// ---- upward pass: q-hat_i = q|_hat + H^T q|_check ------------------------
// A[t][a] = H[a][t] at H[a*k + t] (column-major in t); Bv row a = grid row
// sel[k+a].  Grid rows and output rows are disjoint slot ranges of one
// buffer, passed as separate read and write views.
template <class T, int W>
__global__ void __launch_bounds__(MV_NT *W) k_mv_up(SweepArgs A, const T *__restrict__ qin,
                                                    T *__restrict__ qout, int RP) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T red[(W > 1 ? W - 1 : 1) * MV_TILES * 4 * MV_NT];
  const int i = A.nb + blockIdx.x;
  if (i >= A.ne) return;
  const int m = A.m[i], k = A.k[i];
  if (k == 0) return;
  const int w = threadIdx.x / MV_NT;
  const int l = threadIdx.x & (MV_NT - 1), lr = l & 15, lk = l >> 4;
  const int col = blockIdx.y * 16 + lr;
  const T *g = qin + A.gbeg[i] * RP;
  T *out = qout + A.hbeg[i] * RP;
  const int *sel = A.sel + A.selo[i];
  const T *H = (const T *)A.G + A.go[i];
  const int nr = m - k;
  for (int t0 = 0; t0 < k; t0 += 16 * MV_TILES) {
    acc_t acc[MV_TILES];
#pragma unroll
    for (int tt = 0; tt < MV_TILES; tt++) acc[tt] = acc_t{0, 0, 0, 0};
    for (int a0 = 16 * w; a0 < nr; a0 += 16 * W) {
      int srow[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int a = a0 + 4 * u + lk;
        srow[u] = a < nr ? sel[k + a] : 0;
      }
      T bv[4], av[4][MV_TILES];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int a = a0 + 4 * u + lk;
        const bool ka = a < nr;
        bv[u] = ka ? g[(int64_t)srow[u] * RP + col] : (T)0;
#pragma unroll
        for (int tt = 0; tt < MV_TILES; tt++) {
          const int t = t0 + tt * 16 + lr;
          av[u][tt] = (ka && t < k) ? H[(int64_t)a * k + t] : (T)0;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; u++)
#pragma unroll
        for (int tt = 0; tt < MV_TILES; tt++) acc[tt] = Mfma<T>::op(av[u][tt], bv[u], acc[tt]);
    }
    if (W > 1) reduce_waves<T, W>(acc, red);
    if (w == 0)
#pragma unroll
      for (int tt = 0; tt < MV_TILES; tt++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int t = t0 + tt * 16 + Mfma<T>::row(lk, e);
          if (t < k) out[(int64_t)t * RP + col] = acc[tt][e] + g[(int64_t)sel[t] * RP + col];
        }
  }
}

// ---- coupling: z-hat_i = sum over the L row of i of B_ij q-hat_j ---------
struct CouplingArgs {
  int i0, nnodes;
  const int *Lrow, *Lj;
  const int64_t *boff;
  const int *krow, *kcol;
  const int64_t *hrow, *hcol;
  const void *B;
  int xrun;
};

// The coupling product over row nodes [1, nnodes): run(n0, n1) contracts
// the blocks of row nodes [n0, n1) with ca.B as the block base.  Stored
// blocks: one call.  Evaluated blocks: per chunk of pairs, the chunk's
// blocks are first written to the workspace (placed so that block p sits at
// base + boff[p], as in the stored layout), then contracted.
template <class Run>
static void coupling_chunks(Handle &h, CouplingArgs &ca, size_t es, hipStream_t s, Run run) {
  if (!h.coupling_eval) {
    ca.B = h.B;
    run(1, (int)h.nnodes);
    return;
  }
  for (size_t c = 0; c + 1 < h.cchunk_node.size(); c++) {
    const int n0 = std::max(h.cchunk_node[c], 1), n1 = h.cchunk_node[c + 1];
    if (n1 <= n0 || h.cchunk_ent[c + 1] <= h.cchunk_ent[c]) continue;
    void *base = (char *)h.Bws - es * (size_t)h.cchunk_ent[c];
    eval_coupling_range(h, h.cchunk_pair[c], h.cchunk_pair[c + 1], base, s);
    ca.B = base;
    run(n0, n1);
  }
}

// Workgroups are dealt to the eight XCDs round-robin.  This maps them so
// that each XCD (and its L2) takes runs of `run` consecutive items --
// spatial neighbours in the tree order, which read the same vector rows --
// while the runs still interleave over the XCDs in item order, which keeps
// the levels (and so the work) balanced between them.  The run length is a
// launch-shape option (mv_xcd_run); fewer than 8 * run items map 1:1.
__device__ __forceinline__ int item_of_block(int b, int nitems, int run) {
  if (nitems < 8 * run) return b;
  const int q = b >> 3;
  return (q / run) * (8 * run) + (b & 7) * run + q % run;
}
static inline int xcd_grid(int nitems, int run) {
  return nitems < 8 * run ? nitems : (nitems + 8 * run - 1) / (8 * run) * (8 * run);
}

// Sum of the W partial accumulator tiles of a workgroup into wave 0.
template <class T, int W, int NA>
__device__ __forceinline__ void reduce_waves_n(typename Mfma<T>::acc_t *acc, T *red) {
  const int w = threadIdx.x / MV_NT, l = threadIdx.x & (MV_NT - 1);
  __syncthreads();
  if (w > 0)
#pragma unroll
    for (int x = 0; x < NA; x++)
#pragma unroll
      for (int e = 0; e < 4; e++) red[(((w - 1) * NA + x) * 4 + e) * MV_NT + l] = acc[x][e];
  __syncthreads();
  if (w == 0)
#pragma unroll
    for (int x = 0; x < NA; x++)
#pragma unroll
      for (int e = 0; e < 4; e++)
        for (int v = 0; v < W - 1; v++) acc[x][e] += red[((v * NA + x) * 4 + e) * MV_NT + l];
}

constexpr int MV_WAVES = 4;  // wavefronts per node in the coupling and near products

// 16-row tiles per pass, keeping the operands within 128 registers: the
// coupling product four (FP64 with more than one column tile, or any with
// three or four: two); the near field two for FP64 (most leaves hold fewer
// than 32 points), else as the coupling product
template <class T, int CT>
struct MvShape {
  static constexpr int TT = (CT >= 3 || (sizeof(T) == 8 && CT >= 2)) ? 2 : 4;
};
template <class T, int CT>
struct NearShape {
  static constexpr int TT = sizeof(T) == 8 ? 2 : MvShape<T, CT>::TT;
};

// ---- coupling: z-hat_i = sum over the L row of i of B_ij q-hat_j ---------
// Stored blocks, or the index-only form (Sec. 1.1: a block is fixed by its
// row and column index sets; Sec. 2.3 end) with no block stored: each lane
// then computes the entry B_ij(t, s) = kappa(x_t, y_s) it feeds to the
// matrix core, from the coordinates of the skeleton slots (gathered once
// per construction), with the same kernel-value function the stored form
// uses.  Both forms run the same kernel in the same order of summation, so
// their products agree bit for bit.  Every entry is read or evaluated once
// per product and feeds CT matrix-core steps (one per 16 right-hand sides).
struct CouplingPts {
  const double *xs, *ys;  // D coordinates per slot: row side (X), column side (Y)
  double diag;
  int f32math;
};

template <class T, int KID, int D>
__device__ __forceinline__ T coupling_entry(const double *xp, const double *yp,
                                            const CouplingPts &P) {
  if (P.f32math) return (T)kernel_f32_t<KID, D>(xp, yp, (float)P.diag);
  return (T)kernel_f64_t<KID, D>(xp, yp, P.diag);
}

// One workgroup per row node i.  Its waves split the row tiles of i (wave
// w: tiles w, w + 4, ..., RTW per pass) and walk every pair of i's L row
// together, so a chunk of 16 rows of q-hat_j (all right-hand sides) and the
// coordinates of its 16 column points are loaded once per workgroup into
// LDS (two buffers; the next chunk's loads are in flight while the current
// one is contracted) and every q-hat value read from LDS feeds RTW matrix-
// core steps.  Each lane evaluates the entries of B_ij it feeds.
template <class T, int RTW, int CT, bool EVAL, int KID, int D, int KC = 16>
__global__ void __launch_bounds__(MV_NT *MV_WAVES, 2)
    k_mv_coupling_rows(CouplingArgs A, CouplingPts P, const T *__restrict__ qh,
                       T *__restrict__ zh, int RP, int nitems) {
  typedef typename Mfma<T>::acc_t acc_t;
  static_assert(KC % 16 == 0, "chunks of whole 16-row groups");
  constexpr int QW = 16 * CT;                   // right-hand sides of a chunk row
  constexpr int QE = KC * QW;                   // values of a chunk (KC rows)
  constexpr int NT = MV_NT * MV_WAVES;
  constexpr int QPT = (QE + NT - 1) / NT;       // staged values per thread
  // row tiles of the pair-split path (nodes of up to 16 TTS rows take it)
  constexpr int TTS = (sizeof(T) == 8 && CT >= 3) ? 1 : MvShape<T, CT>::TT;
  constexpr size_t SH_ROWS = sizeof(T) * 2 * QE + sizeof(double) * 2 * KC * D;
  constexpr size_t SH_PAIRS = sizeof(T) * (MV_WAVES - 1) * TTS * CT * 4 * MV_NT;
  __shared__ __align__(16) unsigned char smem[SH_ROWS > SH_PAIRS ? SH_ROWS : SH_PAIRS];
  const int it = item_of_block(blockIdx.x, nitems, A.xrun);
  if (it >= nitems) return;
  const int i = A.i0 + it;
  const int ki = A.krow[i];
  if (ki == 0) return;
  const int tid = threadIdx.x;
  const int w = tid / MV_NT;
  const int l = tid & (MV_NT - 1), lr = l & 15, lk = l >> 4;
  T *out = zh + A.hrow[i] * RP + lr;
  const double *xi = EVAL ? P.xs + A.hrow[i] * D : nullptr;
  const T *Bv = (const T *)A.B;
  const int p0 = A.Lrow[i], p1 = A.Lrow[i + 1];
  const int nt = (ki + 15) / 16;
  if (nt <= TTS) {
    // small nodes: the waves split the pairs instead (each all row tiles),
    // then their partial sums are added in LDS
    T *red = (T *)smem;
    double xr[TTS][D];
    bool tin[TTS];
#pragma unroll
    for (int tt = 0; tt < TTS; tt++) {
      const int t = 16 * tt + lr;
      tin[tt] = t < ki;
#pragma unroll
      for (int e = 0; e < D; e++) xr[tt][e] = (EVAL && tin[tt]) ? xi[(int64_t)t * D + e] : 0.0;
    }
    acc_t acc[TTS * CT];
#pragma unroll
    for (int x = 0; x < TTS * CT; x++) acc[x] = acc_t{0, 0, 0, 0};
    for (int p = p0 + w; p < p1; p += MV_WAVES) {
      const int j = A.Lj[p];
      const int kj = A.kcol[j];
      const T *qj = qh + A.hcol[j] * RP + lr;
      const double *yj = EVAL ? P.ys + A.hcol[j] * D : nullptr;
      const T *Bp = EVAL ? nullptr : Bv + A.boff[p];
      // K in chunks of 16: the operands of four matrix-core steps are
      // loaded (or evaluated) first, then the steps run
      for (int s0 = 0; s0 < kj; s0 += 16) {
        T bv[4][CT], av[4][TTS];
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int s = s0 + 4 * u + lk;
          const bool ks = s < kj;
#pragma unroll
          for (int c = 0; c < CT; c++) bv[u][c] = ks ? qj[(int64_t)s * RP + 16 * c] : (T)0;
          if constexpr (EVAL) {
            double yc[D];
#pragma unroll
            for (int e = 0; e < D; e++) yc[e] = ks ? yj[(int64_t)s * D + e] : 0.0;
#pragma unroll
            for (int tt = 0; tt < TTS; tt++)
              av[u][tt] = (ks && tin[tt]) ? coupling_entry<T, KID, D>(xr[tt], yc, P) : (T)0;
          } else {
#pragma unroll
            for (int tt = 0; tt < TTS; tt++)
              av[u][tt] = (ks && tin[tt]) ? Bp[(int64_t)s * ki + 16 * tt + lr] : (T)0;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
          if (s0 + 4 * u >= kj) break;  // steps past row kj add only zeros (uniform in the wave)
#pragma unroll
          for (int tt = 0; tt < TTS; tt++)
#pragma unroll
            for (int c = 0; c < CT; c++)
              acc[tt * CT + c] = Mfma<T>::op(av[u][tt], bv[u][c], acc[tt * CT + c]);
        }
      }
    }
    reduce_waves_n<T, MV_WAVES, TTS * CT>(acc, red);
    if (w == 0)
#pragma unroll
      for (int tt = 0; tt < TTS; tt++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int t = 16 * tt + Mfma<T>::row(lk, e);
          if (t < ki)
#pragma unroll
            for (int c = 0; c < CT; c++) out[(int64_t)t * RP + 16 * c] = acc[tt * CT + c][e];
        }
    return;
  }
  T (*qs)[QE] = (T (*)[QE])smem;
  double (*ys)[KC * D] = (double (*)[KC * D])(smem + sizeof(T) * 2 * QE);
  for (int tb = 0; tb < nt; tb += MV_WAVES * RTW) {
    // coordinates of this lane's rows t = 16 (tb + w + 4 tt) + lr
    double xr[RTW][D];
    bool tin[RTW];
#pragma unroll
    for (int tt = 0; tt < RTW; tt++) {
      const int t = 16 * (tb + w + MV_WAVES * tt) + lr;
      tin[tt] = t < ki;
#pragma unroll
      for (int e = 0; e < D; e++) xr[tt][e] = (EVAL && tin[tt]) ? xi[(int64_t)t * D + e] : 0.0;
    }
    acc_t acc[RTW * CT];
#pragma unroll
    for (int x = 0; x < RTW * CT; x++) acc[x] = acc_t{0, 0, 0, 0};
    // the chunks of the L row: pair p, rows s0 .. s0 + 15 of q-hat_j
    int p = p0, s0 = 0;
    T qv[QPT];
    double yv = 0.0;
    auto fetch = [&](int pp, int ss) {
      const int j = A.Lj[pp];
      const int kj = A.kcol[j];
      const T *qj = qh + A.hcol[j] * RP;
#pragma unroll
      for (int e = 0; e < QPT; e++) {
        const int q = tid + NT * e;
        const int r = q / QW, cc = q - r * QW;
        qv[e] = (q < QE && ss + r < kj) ? qj[(int64_t)(ss + r) * RP + cc] : (T)0;
      }
      if (EVAL && tid < KC * D) {
        const int r = tid / D;
        yv = ss + r < kj ? P.ys[(A.hcol[j] + ss + r) * D + (tid - r * D)] : 0.0;
      }
    };
    if (p < p1) fetch(p, s0);
    int buf = 0;
    while (p < p1) {
      const int kj = A.kcol[A.Lj[p]];
#pragma unroll
      for (int e = 0; e < QPT; e++) {
        const int q = tid + NT * e;
        if (q < QE) qs[buf][q] = qv[e];
      }
      if (EVAL && tid < KC * D) ys[buf][tid] = yv;
      __syncthreads();
      const T *Bp = EVAL ? nullptr : Bv + A.boff[p];
      // the next chunk's loads, in flight during this chunk's steps
      int pn = p, sn = s0 + KC;
      if (sn >= kj) {
        pn = p + 1;
        sn = 0;
      }
      if (pn < p1) fetch(pn, sn);
      const T *qb = qs[buf];
      const double *yb = ys[buf];
#pragma unroll
      for (int u = 0; u < KC / 4; u++) {
        // steps wholly past row kj of q-hat_j would add only zeros: skipped
        // (the same in every wave, which all walk this pair)
        if (s0 + 4 * u >= kj) break;
        const int sr = 4 * u + lk;  // row of the chunk
        const bool ks = s0 + sr < kj;
        T bv[CT];
#pragma unroll
        for (int c = 0; c < CT; c++) bv[c] = qb[sr * QW + 16 * c + lr];
        double yc[D];
#pragma unroll
        for (int e = 0; e < D; e++) yc[e] = yb[sr * D + e];
#pragma unroll
        for (int tt = 0; tt < RTW; tt++) {
          if (tb + w + MV_WAVES * tt >= nt) break;  // no such tile (uniform in the wave)
          T av = (T)0;
          if (ks && tin[tt]) {
            if constexpr (EVAL)
              av = coupling_entry<T, KID, D>(xr[tt], yc, P);
            else  // stored column-major: entry (t, s) at s ki + t
              av = Bp[(int64_t)(s0 + sr) * ki + 16 * (tb + w + MV_WAVES * tt) + lr];
          }
#pragma unroll
          for (int c = 0; c < CT; c++) acc[tt * CT + c] = Mfma<T>::op(av, bv[c], acc[tt * CT + c]);
        }
      }
      buf ^= 1;
      p = pn;
      s0 = sn;
    }
#pragma unroll
    for (int tt = 0; tt < RTW; tt++) {
      const int t0 = 16 * (tb + w + MV_WAVES * tt);
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int t = t0 + Mfma<T>::row(lk, e);
        if (t < ki)
#pragma unroll
          for (int c = 0; c < CT; c++) out[(int64_t)t * RP + 16 * c] = acc[tt * CT + c][e];
      }
    }
  }
}

template <class T, int CT, int KID, int D>
static void launch_coupling_eval_kd(const CouplingArgs &ca, const CouplingPts &pts, const T *q,
                                    T *z, int RP, int nitems, hipStream_t s) {
  // four row tiles per wave: one pass covers nodes of up to 256 skeleton points
  // chunks of 32 rows of q-hat_j per barrier where that costs no occupancy
  // (the FP64 1/r form); 16 otherwise.  Each accumulator adds its rows in
  // the same order either way.
  constexpr int KC = (KID == SMASH_KERNEL_INV_R && sizeof(T) == 8) ? 32 : 16;
  k_mv_coupling_rows<T, 4, CT, true, KID, D, KC>
      <<<xcd_grid(nitems, ca.xrun), MV_NT * MV_WAVES, 0, s>>>(ca, pts, q, z, RP, nitems);
  SMASH_CHECK_LAUNCH();
}

template <class T, int CT>
static void launch_coupling_eval(const Handle &h, const CouplingArgs &ca, const CouplingPts &pts,
                                 const T *q, T *z, int RP, int nitems, hipStream_t s) {
#define SMASH_CE(KID, D)                                                           if (h.kid == KID && h.d == D) {                                                    launch_coupling_eval_kd<T, CT, KID, D>(ca, pts, q, z, RP, nitems, s);             return;                                                                        }
  SMASH_CE(SMASH_KERNEL_INV_R, 1) SMASH_CE(SMASH_KERNEL_INV_R, 2) SMASH_CE(SMASH_KERNEL_INV_R, 3)
  SMASH_CE(SMASH_KERNEL_LOG_R, 1) SMASH_CE(SMASH_KERNEL_LOG_R, 2) SMASH_CE(SMASH_KERNEL_LOG_R, 3)
  SMASH_CE(SMASH_KERNEL_EXP_R, 1) SMASH_CE(SMASH_KERNEL_EXP_R, 2) SMASH_CE(SMASH_KERNEL_EXP_R, 3)
  SMASH_CE(SMASH_KERNEL_CAUCHY, 1)
#undef SMASH_CE
  throw Error{SMASH_E_UNSUPPORTED, "kernel and dimension without an evaluated coupling form"};
}

// ---- downward pass: grid rows (=/+=) P [I; G] z-hat_i -----------------------
// A[a][t] = G[a][t] at Gt[t*(m-k) + a]; Bv row t = z-hat row t.
template <class T, int W>
__global__ void __launch_bounds__(MV_NT *W) k_mv_down(SweepArgs A, const T *__restrict__ zin,
                                                      T *__restrict__ zout, int RP) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int i = A.nb + blockIdx.x;
  if (i >= A.ne) return;
  const int m = A.m[i], k = A.k[i];
  if (m == 0) return;
  const bool leaf = A.nchild[i] == 0;
  const int w = threadIdx.x / MV_NT;
  const int l = threadIdx.x & (MV_NT - 1), lr = l & 15, lk = l >> 4;
  const int col = blockIdx.y * 16 + lr;
  T *g = zout + A.gbeg[i] * RP;
  const T *zh = zin + A.hbeg[i] * RP;
  const int *sel = A.sel + A.selo[i];
  const T *Gt = (const T *)A.Gt + A.go[i];
  const int nr = m - k;
  // skeleton rows: grid[sel[t]] (=/+=) z-hat[t]
  for (int t = 4 * w + lk; t < k; t += 4 * W) {
    T *dst = g + (int64_t)sel[t] * RP + col;
    const T v = zh[(int64_t)t * RP + col];
    if (leaf)
      *dst = v;
    else
      *dst += v;
  }
  for (int a0 = 16 * MV_TILES * w; a0 < nr; a0 += 16 * MV_TILES * W) {
    acc_t acc[MV_TILES];
#pragma unroll
    for (int tt = 0; tt < MV_TILES; tt++) acc[tt] = acc_t{0, 0, 0, 0};
    for (int t0 = 0; t0 < k; t0 += 16) {
      T bv[4], av[4][MV_TILES];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int t = t0 + 4 * u + lk;
        const bool kt = t < k;
        bv[u] = kt ? zh[(int64_t)t * RP + col] : (T)0;
#pragma unroll
        for (int tt = 0; tt < MV_TILES; tt++) {
          const int a = a0 + tt * 16 + lr;
          av[u][tt] = (kt && a < nr) ? Gt[(int64_t)t * nr + a] : (T)0;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; u++)
#pragma unroll
        for (int tt = 0; tt < MV_TILES; tt++) acc[tt] = Mfma<T>::op(av[u][tt], bv[u], acc[tt]);
    }
#pragma unroll
    for (int tt = 0; tt < MV_TILES; tt++)
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int a = a0 + tt * 16 + Mfma<T>::row(lk, e);
        if (a < nr) {
          T *dst = g + (int64_t)sel[k + a] * RP + col;
          if (leaf)
            *dst = acc[tt][e];
          else
            *dst += acc[tt][e];
        }
      }
  }
}

// ---- near field + scatter: Z[perm_x] = z + sum_{L^-} B_ij q|_j ------------
struct NearArgs {
  int i0, nnodes;
  const int *nchild, *xb, *xe, *yb, *ye, *perm_x;
  const int *Lmrow, *Lmj;
  const int64_t *nboff;
  const void *Bn;
  int has_far;
  int xrun;
};

template <class T, int TT, int CT>
__global__ void __launch_bounds__(MV_NT *MV_WAVES) k_mv_near_out(NearArgs A,
                                                                 const T *__restrict__ q,
                                                                 const T *__restrict__ z,
                                                                 T *__restrict__ Y, int64_t ldy,
                                                                 int R, int RP, int nitems) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T red[(MV_WAVES - 1) * TT * CT * 4 * MV_NT];
  const int it = item_of_block(blockIdx.x, nitems, A.xrun);
  if (it >= nitems) return;
  const int i = A.i0 + it;
  if (A.nchild[i] != 0) return;
  const int xb = A.xb[i], ni = A.xe[i] - xb;
  const int w = threadIdx.x / MV_NT;
  const int l = threadIdx.x & (MV_NT - 1), lr = l & 15, lk = l >> 4;
  const T *Bv = (const T *)A.Bn;
  const int p0 = A.Lmrow[i], p1 = A.Lmrow[i + 1];
  for (int a0 = 0; a0 < ni; a0 += 16 * TT) {
    acc_t acc[TT * CT];
#pragma unroll
    for (int x = 0; x < TT * CT; x++) acc[x] = acc_t{0, 0, 0, 0};
    for (int p = p0 + w; p < p1; p += MV_WAVES) {
      const int j = A.Lmj[p];
      const int yb = A.yb[j], nj = A.ye[j] - yb;
      const T *Bp = Bv + A.nboff[p];
      const T *qj = q + (int64_t)yb * RP + lr;
      for (int b0 = 0; b0 < nj; b0 += 16) {
        T bv[4][CT], av[4][TT];
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int b = b0 + 4 * u + lk;
          const bool kb = b < nj;
#pragma unroll
          for (int c = 0; c < CT; c++) bv[u][c] = kb ? qj[(int64_t)b * RP + 16 * c] : (T)0;
#pragma unroll
          for (int tt = 0; tt < TT; tt++) {
            const int a = a0 + tt * 16 + lr;
            av[u][tt] = (kb && a < ni) ? Bp[b * ni + a] : (T)0;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
          if (b0 + 4 * u >= nj) break;  // steps past column nj add only zeros (uniform in the wave)
#pragma unroll
          for (int tt = 0; tt < TT; tt++)
#pragma unroll
            for (int c = 0; c < CT; c++)
              acc[tt * CT + c] = Mfma<T>::op(av[u][tt], bv[u][c], acc[tt * CT + c]);
        }
      }
    }
    reduce_waves_n<T, MV_WAVES, TT * CT>(acc, red);
    if (w == 0)
#pragma unroll
      for (int tt = 0; tt < TT; tt++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int a = a0 + tt * 16 + Mfma<T>::row(lk, e);
          if (a < ni) {
            const int64_t yrow = (int64_t)A.perm_x[xb + a] * ldy;
#pragma unroll
            for (int c = 0; c < CT; c++) {
              const int col = 16 * c + lr;
              if (col < R) {
                T v = acc[tt * CT + c][e];
                if (A.has_far) v += z[(int64_t)(xb + a) * RP + col];
                Y[yrow + col] = v;
              }
            }
          }
        }
  }
}

template <class T, int CT>
static void launch_coupling(const CouplingArgs &ca, const T *q, T *z, int RP, int nitems,
                            hipStream_t s) {
  // stored blocks: the same kernel, order of summation and result as the
  // evaluated form
  const CouplingPts none{nullptr, nullptr, 0.0, 0};
  k_mv_coupling_rows<T, 4, CT, false, 0, 1>
      <<<xcd_grid(nitems, ca.xrun), MV_NT * MV_WAVES, 0, s>>>(ca, none, q, z, RP, nitems);
  SMASH_CHECK_LAUNCH();
}

template <class T, int CT>
static void launch_near(const NearArgs &na, const T *q, const T *z, T *Y, int64_t ldy, int R,
                        int RP, int nitems, hipStream_t s) {
  k_mv_near_out<T, NearShape<T, CT>::TT, CT>
      <<<xcd_grid(nitems, na.xrun), MV_NT * MV_WAVES, 0, s>>>(na, q, z, Y, ldy, R, RP, nitems);
  SMASH_CHECK_LAUNCH();
}

// ======================================================================
// BF16 apply: the matrices (H^T, G, B_ij, near blocks) are BF16 in the
// matrix-core operand order, vectors stay FP32 and are rounded to BF16 as
// they enter a 16x16x32 step (eight K entries per lane: lane l feeds
// A[l%16][8(l/16) + j] and Bv[8(l/16) + j][l%16], j < 8; results as in the
// FP32 16x16x4 step, row 4(l/16) + e), accumulation FP32.
// ======================================================================
struct SweepArgsB {
  int nb, ne;
  const int *m, *k, *nchild;
  const int64_t *gbeg, *hbeg, *selo, *gou, *god;
  const int *sel;
  const unsigned short *Gu, *Gd;
};

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 load_bf16x8(const unsigned short *p) {
  return __builtin_bit_cast(bf16x8, *(const uint4 *)p);
}
__device__ __forceinline__ bf16x8 zero_bf16x8() {
  return __builtin_bit_cast(bf16x8, uint4{0u, 0u, 0u, 0u});
}

// up: q-hat_i = q|_hat + H^T q|_check; K = grid rows in chunks of 32 per wave
template <int W>
__global__ void __launch_bounds__(MV_NT *W) k_mvb_up(SweepArgsB A, const float *__restrict__ qin,
                                                     float *__restrict__ qout, int RP) {
  __shared__ float red[(W > 1 ? W - 1 : 1) * MV_TILES * 4 * MV_NT];
  const int i = A.nb + blockIdx.x;
  if (i >= A.ne) return;
  const int m = A.m[i], k = A.k[i];
  if (k == 0) return;
  const int w = threadIdx.x / MV_NT;
  const int l = threadIdx.x & (MV_NT - 1), lr = l & 15, lk = l >> 4;
  const int col = blockIdx.y * 16 + lr;
  const float *g = qin + A.gbeg[i] * RP;
  float *out = qout + A.hbeg[i] * RP;
  const int *sel = A.sel + A.selo[i];
  const unsigned short *H = A.Gu + A.gou[i];
  const int nr = m - k;
  for (int t0 = 0; t0 < k; t0 += 16 * MV_TILES) {
    f32x4 acc[MV_TILES];
#pragma unroll
    for (int tt = 0; tt < MV_TILES; tt++) acc[tt] = f32x4{0, 0, 0, 0};
    for (int a0 = 32 * w; a0 < nr; a0 += 32 * W) {
      const int kb = a0 + 8 * lk;
      float xv[8];
#pragma unroll
      for (int j = 0; j < 8; j++) xv[j] = g[(int64_t)sel[k + (kb + j < nr ? kb + j : 0)] * RP + col];
      bf16x8 bv;
      bf16x8 av[MV_TILES];
#pragma unroll
      for (int tt = 0; tt < MV_TILES; tt++) {
        const int t = t0 + tt * 16 + lr;
        av[tt] = (kb < nr && t < k) ? load_bf16x8(H + ((int64_t)(kb >> 3) * k + t) * 8)
                                    : zero_bf16x8();
      }
#pragma unroll
      for (int j = 0; j < 8; j++) bv[j] = (__bf16)(kb + j < nr ? xv[j] : 0.0f);
#pragma unroll
      for (int tt = 0; tt < MV_TILES; tt++) acc[tt] = mfma_bf16(av[tt], bv, acc[tt]);
    }
    if (W > 1) reduce_waves<float, W>(acc, red);
    if (w == 0)
#pragma unroll
      for (int tt = 0; tt < MV_TILES; tt++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int t = t0 + tt * 16 + 4 * lk + e;
          if (t < k) out[(int64_t)t * RP + col] = acc[tt][e] + g[(int64_t)sel[t] * RP + col];
        }
  }
}

// down: grid rows (=/+=) P [I; G] z-hat_i; K = skeleton index in chunks of 32
template <int W>
__global__ void __launch_bounds__(MV_NT *W) k_mvb_down(SweepArgsB A, const float *__restrict__ zin,
                                                       float *__restrict__ zout, int RP) {
  const int i = A.nb + blockIdx.x;
  if (i >= A.ne) return;
  const int m = A.m[i], k = A.k[i];
  if (m == 0) return;
  const bool leaf = A.nchild[i] == 0;
  const int w = threadIdx.x / MV_NT;
  const int l = threadIdx.x & (MV_NT - 1), lr = l & 15, lk = l >> 4;
  const int col = blockIdx.y * 16 + lr;
  float *g = zout + A.gbeg[i] * RP;
  const float *zh = zin + A.hbeg[i] * RP;
  const int *sel = A.sel + A.selo[i];
  const unsigned short *Gd = A.Gd + A.god[i];
  const int nr = m - k;
  for (int t = 4 * w + lk; t < k; t += 4 * W) {
    float *dst = g + (int64_t)sel[t] * RP + col;
    const float v = zh[(int64_t)t * RP + col];
    if (leaf)
      *dst = v;
    else
      *dst += v;
  }
  for (int a0 = 16 * MV_TILES * w; a0 < nr; a0 += 16 * MV_TILES * W) {
    f32x4 acc[MV_TILES];
#pragma unroll
    for (int tt = 0; tt < MV_TILES; tt++) acc[tt] = f32x4{0, 0, 0, 0};
    for (int t0 = 0; t0 < k; t0 += 32) {
      const int kb = t0 + 8 * lk;
      float xv[8];
#pragma unroll
      for (int j = 0; j < 8; j++) xv[j] = zh[(int64_t)(kb + j < k ? kb + j : 0) * RP + col];
      bf16x8 bv;
      bf16x8 av[MV_TILES];
#pragma unroll
      for (int tt = 0; tt < MV_TILES; tt++) {
        const int a = a0 + tt * 16 + lr;
        av[tt] = (kb < k && a < nr) ? load_bf16x8(Gd + ((int64_t)(kb >> 3) * nr + a) * 8)
                                    : zero_bf16x8();
      }
#pragma unroll
      for (int j = 0; j < 8; j++) bv[j] = (__bf16)(kb + j < k ? xv[j] : 0.0f);
#pragma unroll
      for (int tt = 0; tt < MV_TILES; tt++) acc[tt] = mfma_bf16(av[tt], bv, acc[tt]);
    }
#pragma unroll
    for (int tt = 0; tt < MV_TILES; tt++)
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int a = a0 + tt * 16 + 4 * lk + e;
        if (a < nr) {
          float *dst = g + (int64_t)sel[k + a] * RP + col;
          if (leaf)
            *dst = acc[tt][e];
          else
            *dst += acc[tt][e];
        }
      }
  }
}

// coupling: one workgroup per row node, its waves splitting the pairs, K in
// chunks of 32
template <int TT, int CT>
__global__ void __launch_bounds__(MV_NT *MV_WAVES) k_mvb_coupling(CouplingArgs A,
                                                                  const float *__restrict__ qh,
                                                                  float *__restrict__ zh, int RP,
                                                                  int nitems) {
  __shared__ float red[(MV_WAVES - 1) * TT * CT * 4 * MV_NT];
  const int it = item_of_block(blockIdx.x, nitems, A.xrun);
  if (it >= nitems) return;
  const int i = A.i0 + it;
  const int ki = A.krow[i];
  if (ki == 0) return;
  const int w = threadIdx.x / MV_NT;
  const int l = threadIdx.x & (MV_NT - 1), lr = l & 15, lk = l >> 4;
  float *out = zh + A.hrow[i] * RP + lr;
  const unsigned short *Bv = (const unsigned short *)A.B;
  const int p0 = A.Lrow[i], p1 = A.Lrow[i + 1];
  for (int t0 = 0; t0 < ki; t0 += 16 * TT) {
    f32x4 acc[TT * CT];
#pragma unroll
    for (int x = 0; x < TT * CT; x++) acc[x] = f32x4{0, 0, 0, 0};
    for (int p = p0 + w; p < p1; p += MV_WAVES) {
      const int j = A.Lj[p];
      const int kj = A.kcol[j];
      const unsigned short *Bp = Bv + A.boff[p];
      const float *qj = qh + A.hcol[j] * RP + lr;
      for (int s0 = 0; s0 < kj; s0 += 32) {
        const int kb = s0 + 8 * lk;
        float xv[CT][8];
#pragma unroll
        for (int c = 0; c < CT; c++)
#pragma unroll
          for (int jj = 0; jj < 8; jj++)
            xv[c][jj] = qj[(int64_t)(kb + jj < kj ? kb + jj : 0) * RP + 16 * c];
        bf16x8 bv[CT], av[TT];
#pragma unroll
        for (int tt = 0; tt < TT; tt++) {
          const int t = t0 + tt * 16 + lr;
          av[tt] = (kb < kj && t < ki) ? load_bf16x8(Bp + ((kb >> 3) * ki + t) * 8) : zero_bf16x8();
        }
        // vector rows are loaded unconditionally (index clamped into the
        // block) and masked when converted, so no load waits on a branch
#pragma unroll
        for (int c = 0; c < CT; c++)
#pragma unroll
          for (int jj = 0; jj < 8; jj++) bv[c][jj] = (__bf16)(kb + jj < kj ? xv[c][jj] : 0.0f);
#pragma unroll
        for (int tt = 0; tt < TT; tt++)
#pragma unroll
          for (int c = 0; c < CT; c++) acc[tt * CT + c] = mfma_bf16(av[tt], bv[c], acc[tt * CT + c]);
      }
    }
    reduce_waves_n<float, MV_WAVES, TT * CT>(acc, red);
    if (w == 0)
#pragma unroll
      for (int tt = 0; tt < TT; tt++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int t = t0 + tt * 16 + 4 * lk + e;
          if (t < ki)
#pragma unroll
            for (int c = 0; c < CT; c++) out[(int64_t)t * RP + 16 * c] = acc[tt * CT + c][e];
        }
  }
}

// near field + scatter: as k_mv_near_out, K in chunks of 32
template <int TT, int CT>
__global__ void __launch_bounds__(MV_NT *MV_WAVES) k_mvb_near_out(NearArgs A,
                                                                  const float *__restrict__ q,
                                                                  const float *__restrict__ z,
                                                                  float *__restrict__ Y,
                                                                  int64_t ldy, int R, int RP,
                                                                  int nitems) {
  __shared__ float red[(MV_WAVES - 1) * TT * CT * 4 * MV_NT];
  const int it = item_of_block(blockIdx.x, nitems, A.xrun);
  if (it >= nitems) return;
  const int i = A.i0 + it;
  if (A.nchild[i] != 0) return;
  const int xb = A.xb[i], ni = A.xe[i] - xb;
  const int w = threadIdx.x / MV_NT;
  const int l = threadIdx.x & (MV_NT - 1), lr = l & 15, lk = l >> 4;
  const unsigned short *Bv = (const unsigned short *)A.Bn;
  const int p0 = A.Lmrow[i], p1 = A.Lmrow[i + 1];
  for (int a0 = 0; a0 < ni; a0 += 16 * TT) {
    f32x4 acc[TT * CT];
#pragma unroll
    for (int x = 0; x < TT * CT; x++) acc[x] = f32x4{0, 0, 0, 0};
    for (int p = p0 + w; p < p1; p += MV_WAVES) {
      const int j = A.Lmj[p];
      const int yb = A.yb[j], nj = A.ye[j] - yb;
      const unsigned short *Bp = Bv + A.nboff[p];
      const float *qj = q + (int64_t)yb * RP + lr;
      for (int b0 = 0; b0 < nj; b0 += 32) {
        const int kb = b0 + 8 * lk;
        float xv[CT][8];
#pragma unroll
        for (int c = 0; c < CT; c++)
#pragma unroll
          for (int jj = 0; jj < 8; jj++)
            xv[c][jj] = qj[(int64_t)(kb + jj < nj ? kb + jj : 0) * RP + 16 * c];
        bf16x8 bv[CT], av[TT];
#pragma unroll
        for (int tt = 0; tt < TT; tt++) {
          const int a = a0 + tt * 16 + lr;
          av[tt] = (kb < nj && a < ni) ? load_bf16x8(Bp + ((kb >> 3) * ni + a) * 8) : zero_bf16x8();
        }
#pragma unroll
        for (int c = 0; c < CT; c++)
#pragma unroll
          for (int jj = 0; jj < 8; jj++) bv[c][jj] = (__bf16)(kb + jj < nj ? xv[c][jj] : 0.0f);
#pragma unroll
        for (int tt = 0; tt < TT; tt++)
#pragma unroll
          for (int c = 0; c < CT; c++) acc[tt * CT + c] = mfma_bf16(av[tt], bv[c], acc[tt * CT + c]);
      }
    }
    reduce_waves_n<float, MV_WAVES, TT * CT>(acc, red);
    if (w == 0)
#pragma unroll
      for (int tt = 0; tt < TT; tt++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int a = a0 + tt * 16 + 4 * lk + e;
          if (a < ni) {
            const int64_t yrow = (int64_t)A.perm_x[xb + a] * ldy;
#pragma unroll
            for (int c = 0; c < CT; c++) {
              const int col = 16 * c + lr;
              if (col < R) {
                float v = acc[tt * CT + c][e];
                if (A.has_far) v += z[(int64_t)(xb + a) * RP + col];
                Y[yrow + col] = v;
              }
            }
          }
        }
  }
}

template <int CT>
static void launch_bf16_blocks(const CouplingArgs *ca, const NearArgs *na, const float *q,
                               float *z, float *Y, int64_t ldy, int R, int RP, int nitems,
                               hipStream_t s) {
  constexpr int TT = CT >= 3 ? 2 : 4;
  if (ca)
    k_mvb_coupling<TT, CT>
        <<<xcd_grid(nitems, ca->xrun), MV_NT * MV_WAVES, 0, s>>>(*ca, q, z, RP, nitems);
  else
    k_mvb_near_out<TT, CT>
        <<<xcd_grid(nitems, na->xrun), MV_NT * MV_WAVES, 0, s>>>(*na, q, z, Y, ldy, R, RP, nitems);
  SMASH_CHECK_LAUNCH();
}

static void matvec_chunk_bf16(Handle &h, const float *X, int64_t ldx, int R, float *Y,
                              int64_t ldy, float *q, float *z, hipStream_t s) {
  Side &Rw = h.row, &Cl = *h.col;
  const int RP = (R + 15) / 16 * 16;
  const int ct = RP / 16;
  {
    PhaseTimer pt(h, SMASH_PHASE_MV_GATHER, s);
    k_mv_gather<float><<<ceil_div(h.ny * RP, 256), 256, 0, s>>>(X, ldx, h.perm_y, h.ny, R, RP, q);
    SMASH_CHECK_LAUNCH();
  }
  auto blocks = [&](const CouplingArgs *ca, const NearArgs *na, int nitems) {
    switch (ct) {
      case 1: launch_bf16_blocks<1>(ca, na, q, z, Y, ldy, R, RP, nitems, s); break;
      case 2: launch_bf16_blocks<2>(ca, na, q, z, Y, ldy, R, RP, nitems, s); break;
      case 3: launch_bf16_blocks<3>(ca, na, q, z, Y, ldy, R, RP, nitems, s); break;
      default: launch_bf16_blocks<4>(ca, na, q, z, Y, ldy, R, RP, nitems, s); break;
    }
  };
  const bool has_far = h.nlevels >= 2;
  if (has_far) {
    {
      PhaseTimer pt(h, SMASH_PHASE_MV_UP, s);
      for (int l = h.nlevels; l >= 2; l--) {
        const int nb = h.level_beg[l - 1], ne = h.level_beg[l];
        const LevelSide &L = Cl.lv[l];
        SweepArgsB sa{nb, ne, Cl.m, Cl.k, h.nchild, Cl.gbeg, Cl.hbeg, Cl.selo, Cl.gobu, Cl.gobd,
                      L.sel, L.Gbu, L.Gbd};
        const bool split = ne - nb <= h.mv_split_nodes;
        auto up = [&](int nodes) {
          if (split)
            k_mvb_up<4><<<dim3(nodes, ct), 4 * MV_NT, 0, s>>>(sa, q, q, RP);
          else
            k_mvb_up<1><<<dim3(nodes, ct), MV_NT, 0, s>>>(sa, q, q, RP);
          SMASH_CHECK_LAUNCH();
        };
        if (h.batched) {
          up(ne - nb);
        } else {
          for (int i = nb; i < ne; i++) {
            sa.nb = i;
            sa.ne = i + 1;
            up(1);
          }
        }
      }
    }
    CouplingArgs ca{1, h.nnodes, h.Lrow, h.Lj, h.boff, Rw.k, Cl.k, Rw.hbeg, Cl.hbeg, h.B,
                    h.mv_xcd_run};
    {
      PhaseTimer pt(h, SMASH_PHASE_MV_COUPLING, s);
      coupling_chunks(h, ca, sizeof(unsigned short), s, [&](int n0, int n1) {
        if (h.batched) {
          ca.i0 = n0;
          blocks(&ca, nullptr, n1 - n0);
        } else {
          for (int i = n0; i < n1; i++) {
            ca.i0 = i;
            blocks(&ca, nullptr, 1);
          }
        }
      });
    }
    PhaseTimer pt(h, SMASH_PHASE_MV_DOWN, s);
    for (int l = 2; l <= h.nlevels; l++) {
      const int nb = h.level_beg[l - 1], ne = h.level_beg[l];
      const LevelSide &L = Rw.lv[l];
      SweepArgsB sa{nb, ne, Rw.m, Rw.k, h.nchild, Rw.gbeg, Rw.hbeg, Rw.selo, Rw.gobu, Rw.gobd,
                    L.sel, L.Gbu, L.Gbd};
      const bool split = ne - nb <= h.mv_split_nodes;
      auto down = [&](int nodes) {
        if (split)
          k_mvb_down<4><<<dim3(nodes, ct), 4 * MV_NT, 0, s>>>(sa, z, z, RP);
        else
          k_mvb_down<1><<<dim3(nodes, ct), MV_NT, 0, s>>>(sa, z, z, RP);
        SMASH_CHECK_LAUNCH();
      };
      if (h.batched) {
        down(ne - nb);
      } else {
        for (int i = nb; i < ne; i++) {
          sa.nb = i;
          sa.ne = i + 1;
          down(1);
        }
      }
    }
  }
  NearArgs na{0, h.nnodes, h.nchild, h.xb, h.xe, h.yb, h.ye, h.perm_x, h.Lmrow, h.Lmj, h.nboff,
              h.Bn, has_far ? 1 : 0, h.mv_xcd_run};
  PhaseTimer pt(h, SMASH_PHASE_MV_NEAR_OUT, s);
  if (h.batched) {
    blocks(nullptr, &na, h.nnodes);
  } else {
    for (int i = 0; i < h.nnodes; i++) {
      na.i0 = i;
      blocks(nullptr, &na, 1);
    }
  }
}

template <class T>
static void matvec_chunk(Handle &h, const T *X, int64_t ldx, int R, T *Y, int64_t ldy, T *q,
                         T *z, hipStream_t s) {
  Side &Rw = h.row, &Cl = *h.col;
  const bool f64 = h.apply_prec == SMASH_F64;
  const int RP = (R + 15) / 16 * 16;
  const int ct = RP / 16;
  {
    PhaseTimer pt(h, SMASH_PHASE_MV_GATHER, s);
    k_mv_gather<T><<<ceil_div(h.ny * RP, 256), 256, 0, s>>>(X, ldx, h.perm_y, h.ny, R, RP, q);
    SMASH_CHECK_LAUNCH();
  }
  const bool has_far = h.nlevels >= 2;
  {
    PhaseTimer pt(h, SMASH_PHASE_MV_UP, s);
    for (int l = h.nlevels; l >= 2; l--) {
      int nb = h.level_beg[l - 1], ne = h.level_beg[l];
      const LevelSide &L = Cl.lv[l];
      SweepArgs sa{nb, ne, Cl.m, Cl.k, h.nchild, Cl.gbeg, Cl.hbeg, Cl.selo, Cl.go, L.sel,
                   f64 ? (const void *)L.G : (const void *)L.G32,
                   f64 ? (const void *)L.Gt : (const void *)L.Gt32};
      // few nodes with long grids: split each node over four waves (the
      // plain form uses the same shape per level, so both round alike)
      const bool split = ne - nb <= h.mv_split_nodes;
      auto up = [&](int nodes) {
        if (split)
          k_mv_up<T, 4><<<dim3(nodes, ct), 4 * MV_NT, 0, s>>>(sa, q, q, RP);
        else
          k_mv_up<T, 1><<<dim3(nodes, ct), MV_NT, 0, s>>>(sa, q, q, RP);
        SMASH_CHECK_LAUNCH();
      };
      if (h.batched) {
        up(ne - nb);
      } else {
        for (int i = nb; i < ne; i++) {
          sa.nb = i;
          sa.ne = i + 1;
          up(1);
        }
      }
    }
  }
  if (has_far) {
    CouplingArgs ca{1, h.nnodes, h.Lrow, h.Lj, h.boff, Rw.k, Cl.k, Rw.hbeg, Cl.hbeg, h.B,
                    h.mv_xcd_run};
    {
      PhaseTimer pt(h, SMASH_PHASE_MV_COUPLING, s);
      auto coupling = [&](int nitems) {
        switch (ct) {
          case 1: launch_coupling<T, 1>(ca, q, z, RP, nitems, s); break;
          case 2: launch_coupling<T, 2>(ca, q, z, RP, nitems, s); break;
          case 3: launch_coupling<T, 3>(ca, q, z, RP, nitems, s); break;
          default: launch_coupling<T, 4>(ca, q, z, RP, nitems, s); break;
        }
      };
      if (h.coupling_fused) {
        const CouplingPts pts{h.xs_slot, h.ys_slot, h.diag, h.eval_prec == SMASH_F32 ? 1 : 0};
        auto fused = [&](int nitems) {
          switch (ct) {
            case 1: launch_coupling_eval<T, 1>(h, ca, pts, q, z, RP, nitems, s); break;
            case 2: launch_coupling_eval<T, 2>(h, ca, pts, q, z, RP, nitems, s); break;
            case 3: launch_coupling_eval<T, 3>(h, ca, pts, q, z, RP, nitems, s); break;
            default: launch_coupling_eval<T, 4>(h, ca, pts, q, z, RP, nitems, s); break;
          }
        };
        if (h.batched) {
          ca.i0 = 1;
          fused((int)h.nnodes - 1);
        } else {
          for (int i = 1; i < h.nnodes; i++) {
            ca.i0 = i;
            fused(1);
          }
        }
      } else {
        coupling_chunks(h, ca, sizeof(T), s, [&](int n0, int n1) {
          if (h.batched) {
            ca.i0 = n0;
            coupling(n1 - n0);
          } else {
            for (int i = n0; i < n1; i++) {
              ca.i0 = i;
              coupling(1);
            }
          }
        });
      }
    }
    PhaseTimer pt(h, SMASH_PHASE_MV_DOWN, s);
    for (int l = 2; l <= h.nlevels; l++) {
      int nb = h.level_beg[l - 1], ne = h.level_beg[l];
      const LevelSide &L = Rw.lv[l];
      SweepArgs sa{nb, ne, Rw.m, Rw.k, h.nchild, Rw.gbeg, Rw.hbeg, Rw.selo, Rw.go, L.sel,
                   f64 ? (const void *)L.G : (const void *)L.G32,
                   f64 ? (const void *)L.Gt : (const void *)L.Gt32};
      const bool split = ne - nb <= h.mv_split_nodes;
      auto down = [&](int nodes) {
        if (split)
          k_mv_down<T, 4><<<dim3(nodes, ct), 4 * MV_NT, 0, s>>>(sa, z, z, RP);
        else
          k_mv_down<T, 1><<<dim3(nodes, ct), MV_NT, 0, s>>>(sa, z, z, RP);
        SMASH_CHECK_LAUNCH();
      };
      if (h.batched) {
        down(ne - nb);
      } else {
        for (int i = nb; i < ne; i++) {
          sa.nb = i;
          sa.ne = i + 1;
          down(1);
        }
      }
    }
  }
  NearArgs na{0, h.nnodes, h.nchild, h.xb, h.xe, h.yb, h.ye, h.perm_x, h.Lmrow, h.Lmj, h.nboff,
              h.Bn, has_far ? 1 : 0, h.mv_xcd_run};
  {
    PhaseTimer pt(h, SMASH_PHASE_MV_NEAR_OUT, s);
    auto near = [&](int nitems) {
      switch (ct) {
        case 1: launch_near<T, 1>(na, q, z, Y, ldy, R, RP, nitems, s); break;
        case 2: launch_near<T, 2>(na, q, z, Y, ldy, R, RP, nitems, s); break;
        case 3: launch_near<T, 3>(na, q, z, Y, ldy, R, RP, nitems, s); break;
        default: launch_near<T, 4>(na, q, z, Y, ldy, R, RP, nitems, s); break;
      }
    };
    if (h.batched) {
      near(h.nnodes);
    } else {
      for (int i = 0; i < h.nnodes; i++) {
        na.i0 = i;
        near(1);
      }
    }
  }
}

// Workspace: q and z in slot space, 64 right-hand sides per pass.  Returns
// true when it was (re)allocated, which invalidates captured graphs.
static bool ensure_workspace(Handle &h, int nrhs, hipStream_t s) {
  const int RC = 64;
  const int chunk = nrhs < RC ? nrhs : RC;
  const int cp = (chunk + 15) / 16 * 16;
  if (h.ws_nrhs >= cp) return false;
  // the captured products hold the old buffers: they go first
  drop_graphs(h);
  // earlier products (on any stream) may still read the old buffers: wait
  // for the last of them (they are ordered by prod_done), then give the
  // buffers back as idle memory
  if (h.prod_done && h.ws_nrhs > 0) SMASH_HIP(hipEventSynchronize(h.prod_done));
  h.ws_mem.release(true);
  h.ws_nrhs = 0;  // (a failed allocation below leaves no buffer behind)
  h.qbuf = h.zbuf = nullptr;
  h.ws_mem.stream = s;
  h.qbuf = h.ws_mem.alloc(sizeof(double) * (size_t)h.col->nslots * cp);
  h.zbuf = h.ws_mem.alloc(sizeof(double) * (size_t)h.row.nslots * cp);
  h.ws_nrhs = cp;
  return true;
}

template <class T>
static void matvec_t(Handle &h, const T *X, int64_t ldx, int nrhs, T *Y, int64_t ldy, T *q, T *z,
                     int chunk, hipStream_t s) {
  for (int c0 = 0; c0 < nrhs; c0 += chunk) {
    const int R = nrhs - c0 < chunk ? nrhs - c0 : chunk;
    if (h.apply_prec == SMASH_BF16)
      matvec_chunk_bf16(h, (const float *)(X + c0), ldx, R, (float *)(Y + c0), ldy, (float *)q,
                        (float *)z, s);
    else
      matvec_chunk<T>(h, X + c0, ldx, R, Y + c0, ldy, q, z, s);
  }
}

// q and z (slot-space vectors of the column and row side) and the number of
// right-hand sides per pass through the tree
static void launch_sequence_in(Handle &h, const void *X, int64_t ldx, int nrhs, void *Y,
                               int64_t ldy, void *q, void *z, int chunk, hipStream_t s) {
  if (h.apply_prec == SMASH_F64)
    matvec_t<double>(h, (const double *)X, ldx, nrhs, (double *)Y, ldy, (double *)q,
                     (double *)z, chunk, s);
  else
    matvec_t<float>(h, (const float *)X, ldx, nrhs, (float *)Y, ldy, (float *)q, (float *)z,
                    chunk, s);
}

static void launch_sequence(Handle &h, const void *X, int64_t ldx, int nrhs, void *Y,
                            int64_t ldy, hipStream_t s) {
  const int RC = 64;  // right-hand sides per pass through the tree
  launch_sequence_in(h, X, ldx, nrhs, Y, ldy, h.qbuf, h.zbuf, nrhs < RC ? nrhs : RC, s);
}

// An executable graph is destroyed once its last launch has completed.
static void destroy_graph(GraphEntry &g) {
  if (g.done) {
    (void)hipEventSynchronize(g.done);
    (void)hipEventDestroy(g.done);
  }
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g.done = nullptr;
  g.exec = nullptr;
}

void drop_graphs(Handle &h) {
  for (auto &g : h.graphs) destroy_graph(g);
  h.graphs.clear();
}

// The product.  Eager launches, or -- with the graphs option and timing off
// -- the same launch sequence captured once into a HIP graph on the second
// call with the same arguments and replayed from then on (one graph launch
// instead of 2 + 2(levels - 1) + 2 kernel launches per 64 right-hand sides).
static void run_matvec_on(Handle &h, const void *X, int64_t ldx, int nrhs, void *Y, int64_t ldy,
                          hipStream_t s);

// Products of one handle share its workspace (and the evaluated form's
// block chunks): one on another stream than the previous product first
// waits for it; each records prod_done at its end.
void run_matvec(Handle &h, const void *X, int64_t ldx, int nrhs, void *Y, int64_t ldy,
                hipStream_t s) {
  if (h.prod_done && h.prod_stream && h.prod_stream != s)
    SMASH_HIP(hipStreamWaitEvent(s, h.prod_done, 0));
  run_matvec_on(h, X, ldx, nrhs, Y, ldy, s);
  if (h.prod_done) {
    SMASH_HIP(hipEventRecord(h.prod_done, s));
    h.prod_stream = s;
  }
}

static void run_matvec_on(Handle &h, const void *X, int64_t ldx, int nrhs, void *Y, int64_t ldy,
                          hipStream_t s) {
  ensure_workspace(h, nrhs, s);
  if (!h.use_graphs || h.timing) {
    launch_sequence(h, X, ldx, nrhs, Y, ldy, s);
    return;
  }
  GraphEntry *e = nullptr;
  for (auto &g : h.graphs)
    if (g.X == X && g.ldx == ldx && g.nrhs == nrhs && g.Y == Y && g.ldy == ldy) e = &g;
  if (!e) {
    if (h.graphs.size() >= 8) {  // keep the eight most recent argument sets
      destroy_graph(h.graphs.front());
      h.graphs.erase(h.graphs.begin());
    }
    h.graphs.push_back(GraphEntry{X, ldx, nrhs, Y, ldy, 0, nullptr, nullptr});
    e = &h.graphs.back();
  }
  e->calls++;
  if (!e->exec && e->calls < 2) {
    launch_sequence(h, X, ldx, nrhs, Y, ldy, s);
    return;
  }
  if (!e->exec) {
    if (!h.cap_stream) SMASH_HIP(hipStreamCreateWithFlags(&h.cap_stream, hipStreamNonBlocking));
    SMASH_HIP(hipStreamBeginCapture(h.cap_stream, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
      launch_sequence(h, X, ldx, nrhs, Y, ldy, h.cap_stream);
    } catch (...) {
      (void)hipStreamEndCapture(h.cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    SMASH_HIP(hipStreamEndCapture(h.cap_stream, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    SMASH_HIP(ie);
    e->exec = ex;
    h.graph_captures++;
  }
  if (!e->done) SMASH_HIP(hipEventCreateWithFlags(&e->done, hipEventDisableTiming));
  SMASH_HIP(hipGraphLaunch(e->exec, s));
  SMASH_HIP(hipEventRecord(e->done, s));
  h.graph_replays++;
}

// ------------------------------------------- Cauchy-like generators
// A Cauchy-like matrix with generators w (nx x p) and v (ny x p) is
// sum_l diag(w_l) C diag(v_l) (eqs. (6.1)-(6.2)).  Each term's HSS generators
// are the handle's with U, D and V scaled by the generator columns, and the
// product of their merged sum is taken here as one product of the handle's
// approximation with the p R columns v_l o X side by side (column l R + r
// holds v_l o X_r), then Y = sum_l w_l o Z_l, the terms added in the order
// l = 0, 1, ...; every column of the stacked product is computed as it
// would be alone.
template <class T>
__global__ void k_cl_stack(const T *X, int64_t ldx, int R, const double *v, int p, int64_t ny,
                           T *Xs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pr = (int64_t)p * R;
  if (e >= ny * pr) return;
  const int64_t j = e / pr;
  const int c = (int)(e - j * pr), l = c / R, r = c - l * R;
  Xs[e] = (T)(v[j * p + l] * (double)X[j * ldx + r]);
}

template <class T>
__global__ void k_cl_combine(const T *Z, int R, const double *w, int p, int64_t nx, T *Y,
                             int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nx * R) return;
  const int64_t i = e / R;
  const int r = (int)(e - i * R);
  const T *zi = Z + i * (int64_t)p * R + r;
  double acc = w[i * p] * (double)zi[0];
  for (int l = 1; l < p; l++) acc = acc + w[i * p + l] * (double)zi[(int64_t)l * R];
  Y[i * ldy + r] = (T)acc;
}

template <class T>
static void cauchy_like_t(Handle &h, const T *X, int64_t ldx, int nrhs, const double *w,
                          const double *v, int p, T *Y, int64_t ldy, hipStream_t s) {
  const int pr = p * nrhs;
  DeviceArena tmp;
  tmp.stream = s;
  try {
    T *Xs = tmp.alloc_n<T>((size_t)h.ny * pr);
    T *Zs = tmp.alloc_n<T>((size_t)h.nx * pr);
    k_cl_stack<T><<<ceil_div(h.ny * pr, 256), 256, 0, s>>>(X, ldx, nrhs, v, p, h.ny, Xs);
    SMASH_CHECK_LAUNCH();
    run_matvec(h, Xs, pr, pr, Zs, pr, s);
    k_cl_combine<T><<<ceil_div(h.nx * nrhs, 256), 256, 0, s>>>(Zs, nrhs, w, p, h.nx, Y, ldy);
    SMASH_CHECK_LAUNCH();
  } catch (...) {
    tmp.release(false);
    throw;
  }
  tmp.release(false);  // stream-ordered: after the combine
}

void run_cauchy_like(Handle &h, const void *X, int64_t ldx, int nrhs, const double *w,
                     const double *v, int p, void *Y, int64_t ldy, hipStream_t s) {
  if (h.apply_prec == SMASH_F64)
    cauchy_like_t<double>(h, (const double *)X, ldx, nrhs, w, v, p, (double *)Y, ldy, s);
  else
    cauchy_like_t<float>(h, (const float *)X, ldx, nrhs, w, v, p, (float *)Y, ldy, s);
}

// ---------------------------------------------- product without allocation
// The product's only device memory beyond the handle, X and Y is its pair of
// slot-space vectors.  For callers that cannot allocate, they come from this
// file-scope array instead of the handle's workspace: one copy per device,
// held until the process ends, shared by every such call on that device.
// In host code `scratch` names a host-side stand-in, not the device array:
// its device address is obtained once per device (noalloc_scratch) and only
// that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[SMASH_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];

// Device address of `scratch` on device dev, looked up on the first call for
// that device with the device current (the caller's device is restored).
static void *noalloc_scratch(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    throw Error{SMASH_E_DEVICE, "device index outside the no-allocation product's table"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    SMASH_HIP(hipGetDevice(&cur));
    if (cur != dev) SMASH_HIP(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      throw Error{SMASH_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e)};
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Columns per pass whose vectors fit in the array: 64, 48, 32 or 16, and no
// more than the right-hand sides rounded up to 16; 0 if 16 do not fit.
static int noalloc_chunk(const Handle &h, int nrhs, size_t *zoff) {
  const size_t es = h.apply_prec == SMASH_F64 ? sizeof(double) : sizeof(float);
  const int rp = (nrhs + 15) / 16 * 16;
  for (int cw = 64; cw >= 16; cw -= 16) {
    if (cw > rp && cw > 16) continue;
    const size_t qb = ((size_t)h.col->nslots * cw * es + 255) / 256 * 256;
    const size_t zb = (size_t)h.row.nslots * cw * es;
    if (qb + zb <= (size_t)SMASH_NOALLOC_SCRATCH_BYTES) {
      *zoff = qb;
      return nrhs < cw ? nrhs : cw;
    }
  }
  return 0;
}

void run_matvec_noalloc(Handle &h, const void *X, int64_t ldx, int nrhs, void *Y, int64_t ldy,
                        hipStream_t s) {
  size_t zoff = 0;
  const int chunk = noalloc_chunk(h, nrhs, &zoff);
  if (chunk == 0) {
    const size_t es = h.apply_prec == SMASH_F64 ? sizeof(double) : sizeof(float);
    throw Error{SMASH_E_INVALID_ARG,
                "the product's vectors need " +
                    std::to_string((size_t)(h.col->nslots + h.row.nslots) * 16 * es) +
                    " bytes at 16 columns; the no-allocation product holds at most " +
                    std::to_string((long long)SMASH_NOALLOC_SCRATCH_BYTES)};
  }
  char *base = (char *)noalloc_scratch(h.device);
  // eager launches only; phase timers would create events
  struct NoTimers {
    Handle &h;
    int saved;
    explicit NoTimers(Handle &h_) : h(h_), saved(h_.timing) { h.timing = 0; }
    ~NoTimers() { h.timing = saved; }
  } nt(h);
  launch_sequence_in(h, X, ldx, nrhs, Y, ldy, base, base + zoff, chunk, s);
}

}  // namespace smash
