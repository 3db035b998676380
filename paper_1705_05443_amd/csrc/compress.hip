// compress.hip -- level-wise construction of the nested bases (Sec. 3.3):
// for l = L, ..., 2 every node of level l, in one launch per phase,
//   * forms its current grid (leaf points, eq. (3.6); else the children's
//     skeletons, eqs. (3.14), (3.18)),
//   * (HSS) takes the truncated SVD of its near-field block row, eqs.
//     (3.7)-(3.8) / (3.11)-(3.12), keeping sigma >= eps_svd * sigma_1,
//   * evaluates the interpolation basis U-hat of eq. (2.2) on the grid
//     (tensor Lagrange basis on first-kind Chebyshev points of its box),
//   * runs compr (eq. (2.14)): strong rank-revealing QR (Thm. 2.4) of
//     M = C^T with C = U-hat or [U-hat, S], giving the skeleton i-hat and
//     G with U = P [I; G] (eq. (2.11)), stored canonically (both index sets
//     ascending).
//
// One workgroup owns one node at a time (persistent grid striding over the
// level's nodes).  Two forms: the register form (k_compr_w) keeps the
// columns of M = C^T in registers for grids of up to 256 points and c <= 64;
// the wide form (k_compr_s) streams them from a column-major tile in LDS or
// in a per-workgroup global scratch.  Column norms for the pivot choice are
// recomputed from the transformed columns after each Householder step (no
// downdating), the arg-max is a DPP reduction, and ties go to the lowest
// position.  All arithmetic is FP64.
#include <algorithm>
#include <mutex>

#include "common.cuh"

namespace smash {

constexpr int ID_CMAX = 512;  // largest basis width c (p^d plus HSS near vectors)
constexpr int ID_PMAX = 64;   // largest interpolation order

struct IdArgs {
  int nb, ne;  // node range
  const double *lo, *hi;
  int d, p, c0;
  const int *m;
  const int64_t *gbeg;
  const int *slot_id;
  const double *P;  // permuted coordinates of this side, n x d
  const int64_t *selo, *go;
  int *sel_out;
  double *G_out;
  int *k_out;
  const double *S;  // HSS near-field vectors, per node m x ks (row-major) at S_off
  const int64_t *S_off;
  const int *ks;
  double tol, f;
  int *swaps;    // total swap count (atomic)
  int *err;      // set to 1 when the swap cap is hit
  int gt_out;    // k_compr_w: write G^T (k x (m-k) row-major) instead of G
  double *G2_out;  // k_compr_w: also the other orientation there (null: not)
  // k_compr_w: with `order`, the nodes order[*ord_lo .. ne - nb) (the rest
  // of a level whose largest grids went to the wide form); else nb .. ne-1
  const int *order, *ord_lo;
  // the column side of the double-layer kernel: basis rows r < c0 are the
  // Lagrange values of row r mod pd times the point's m_1 (r < pd) or m_2
  // (c0 = 2 pd); pd is p^d and pdat the per-point data by point id
  int dlw, pd;
  const double *pdat;
  // > 0: the Taylor basis of eqs. (2.4)-(2.5) (d = 1) with this g in place
  // of the Lagrange basis (see taylor_phi)
  double taylor_g;
};

// phi_q of the Taylor basis (2.4)-(2.5) at x for the box [lo, hi] with
// hi > lo: eta_q (x - a)^q / q! with a the box's center, delta its half
// width and eta_q = (q g / delta)^q, i.e. (u q g)^q / q! for
// u = (x - a) / delta, taken as the running product of (u q g) / k
__device__ __forceinline__ double taylor_phi(double x, double lo, double hi, int q, double g) {
  const double a = 0.5 * (lo + hi), del = 0.5 * (hi - lo);
  const double u = (x - a) / del;
  const double w = u * ((double)q * g);
  double v = 1.0;
  for (int k = 1; k <= q; k++) v = v * w / (double)k;
  return v;
}

// ---- lane exchanges (DPP) ------------------------------------------------
// update_dpp with old = the lane's own value: lanes outside row_mask keep it
template <int CTRL, int ROWM = 0xF>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(x), __double2loint(x), CTRL, ROWM,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(x), __double2hiint(x), CTRL, ROWM,
                                             0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWM = 0xF>
__device__ __forceinline__ int dpp_i32(int x) {
  return __builtin_amdgcn_update_dpp(x, x, CTRL, ROWM, 0xF, false);
}
// the same for permutations in which every lane has a source lane (quad
// permutations, mirrors): no old value to keep, so no copy of x first
template <int CTRL>
__device__ __forceinline__ double perm_f64(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ int perm_i32(int x) {
  return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ double readlane_f64(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}
// sum over the LPC lanes of a group (the same value, bit for bit, in each:
// every lane adds the same two operands)
template <int LPC>
__device__ __forceinline__ double group_sum(double x) {
  if constexpr (LPC >= 2) x += perm_f64<0xB1>(x);  // quad_perm [1,0,3,2]
  if constexpr (LPC >= 4) x += perm_f64<0x4E>(x);  // quad_perm [2,3,0,1]
  return x;
}
template <int LPC>
__device__ __forceinline__ int group_max(int x) {
  if constexpr (LPC >= 2) x = max(x, perm_i32<0xB1>(x));
  if constexpr (LPC >= 4) x = max(x, perm_i32<0x4E>(x));
  return x;
}
// the value of group member HS in every lane of the group
template <int LPC, int HS>
__device__ __forceinline__ double group_bcast(double x) {
  if constexpr (LPC == 1)
    return x;
  else if constexpr (LPC == 2)
    return perm_f64<HS | (HS << 2) | ((2 + HS) << 4) | ((2 + HS) << 6)>(x);
  else
    return perm_f64<HS | (HS << 2) | (HS << 4) | (HS << 6)>(x);
}

// ---- block reductions --------------------------------------------------
struct ArgMax {
  double v;
  int a;
};

// larger value wins; ties: smaller index (NaN never wins)
__device__ inline ArgMax amax_pick(ArgMax x, ArgMax y) {
  if (y.v > x.v || (y.v == x.v && y.a < x.a && y.a >= 0)) return y;
  if (x.a < 0) return y;
  return x;
}

// Index part of an arg-max over the first NL lanes once the maximum v is
// known: the single lane holding it (the usual case, one ballot), else the
// smallest index among the lanes that hold it (DPP minimum over NL lanes).
template <int NL>
__device__ __forceinline__ int argmax_index(ArgMax x, double v, bool valid) {
  const bool on = valid && x.v == v && x.a >= 0;
  const uint64_t hit = __ballot(on);
  if (hit == 0) return -1;
  if (__popcll(hit) == 1) return __builtin_amdgcn_readlane(x.a, __ffsll((unsigned long long)hit) - 1);
  int a = on ? x.a : 0x7fffffff;
  if constexpr (NL > 1) a = min(a, perm_i32<0xB1>(a));
  if constexpr (NL > 2) a = min(a, perm_i32<0x4E>(a));
  if constexpr (NL > 4) a = min(a, perm_i32<0x141>(a));
  if constexpr (NL > 8) a = min(a, perm_i32<0x140>(a));
  if constexpr (NL > 16) {
    a = min(a, dpp_i32<0x142, 0xA>(a));
    a = min(a, dpp_i32<0x143, 0xC>(a));
    return __builtin_amdgcn_readlane(a, WAVE - 1);
  } else {
    return __builtin_amdgcn_readlane(a, 0);
  }
}

// arg-max over the wavefront (all 64 lanes active), returned to every lane:
// the largest value, then the smallest index among the lanes holding it.
// Values are norms (>= 0) or -1 with index -1 for lanes without a
// candidate.  Butterfly steps inside quads, mirrors inside half-rows and
// rows, then the row broadcasts leave the maximum in lane 63.
__device__ inline ArgMax wave_argmax(ArgMax x) {
  double v = x.v;
  v = fmax(v, perm_f64<0xB1>(v));       // quad_perm [1,0,3,2]
  v = fmax(v, perm_f64<0x4E>(v));       // quad_perm [2,3,0,1]
  v = fmax(v, perm_f64<0x141>(v));      // row_half_mirror
  v = fmax(v, perm_f64<0x140>(v));      // row_mirror
  v = fmax(v, dpp_f64<0x142, 0xA>(v));  // row_bcast:15 into rows 1, 3
  v = fmax(v, dpp_f64<0x143, 0xC>(v));  // row_bcast:31 into rows 2, 3
  v = readlane_f64(v, WAVE - 1);
  return ArgMax{v, argmax_index<WAVE>(x, v, true)};
}

// The same when every group of four consecutive lanes holds one candidate
// (the same value and index in its four lanes): the two exchanges inside the
// quads are skipped and the index is taken among the groups' first lanes.
__device__ inline ArgMax wave_argmax_quad(ArgMax x) {
  double v = x.v;
  v = fmax(v, perm_f64<0x141>(v));      // row_half_mirror (lane i and 7 - i: other quads)
  v = fmax(v, perm_f64<0x140>(v));      // row_mirror
  v = fmax(v, dpp_f64<0x142, 0xA>(v));  // row_bcast:15 into rows 1, 3
  v = fmax(v, dpp_f64<0x143, 0xC>(v));  // row_bcast:31 into rows 2, 3
  v = readlane_f64(v, WAVE - 1);
  return ArgMax{v, argmax_index<WAVE>(x, v, (threadIdx.x & 3) == 0)};
}

// the same over the first NL (<= 16) lanes (the per-wave results of a block)
template <int NL>
__device__ inline ArgMax lanes_argmax(ArgMax x) {
  const bool valid = (int)(threadIdx.x & (WAVE - 1)) < NL;
  double v = valid ? x.v : -1.0;
  if constexpr (NL > 1) v = fmax(v, perm_f64<0xB1>(v));
  if constexpr (NL > 2) v = fmax(v, perm_f64<0x4E>(v));
  if constexpr (NL > 4) v = fmax(v, perm_f64<0x141>(v));
  if constexpr (NL > 8) v = fmax(v, perm_f64<0x140>(v));
  v = readlane_f64(v, 0);
  return ArgMax{v, argmax_index<NL>(x, v, valid)};
}

// (NW = wavefronts per workgroup, a compile-time constant: the workgroup
// size read at run time is a load from the dispatch arguments)
template <int NW>
__device__ inline ArgMax block_argmax(ArgMax x, ArgMax *lds) {
  x = wave_argmax(x);
  if constexpr (NW == 1) return x;
  const int wid = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  __syncthreads();
  if (lane == 0) lds[wid] = x;
  __syncthreads();
  return lanes_argmax<NW>(lane < NW ? lds[lane] : ArgMax{-1.0, -1});
}

template <int NW>
__device__ inline double block_sum(double v, double *lds) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  const int wid = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < NW; w++) r += lds[w];
  return r;
}

// ------------------------------------------------------------------------
// Register-resident compr for nodes whose grid fits one workgroup and whose
// basis width fits CMAX.  Columns of M = C^T are held in registers for the
// whole algorithm, in groups of LPC consecutive lanes: a group owns J grid
// columns (a = J cb + j) and lane phase h of the group keeps their rows
// r = LPC u + h (u < CMAX / LPC).  Each value read from LDS (a reflector
// entry, an entry of R11) then feeds J columns, and sums over a column are
// lane exchanges (DPP) inside the group.  So
//   * a Householder step is one block arg-max of the squared residual norms
//     (one barrier: each wavefront's own winner stages its column in LDS
//     beforehand), the reflector v read from the winning slot (v^T v follows
//     from the pivot norm as 2 beta (beta + |x_t|)), and a register update of
//     every column (scale 0 for the pivot and finished ones) with the squared
//     norms of the remaining ones recomputed;
//   * a column's position (the order the QR works in) is a label: a pivot
//     or a Gu-Eisenstat swap relabels two columns instead of moving data,
//     and ties still go to the lowest current position;
//   * the swap test solves R11 in every column at once, by column-oriented
//     back substitution against R11 in LDS padded to [R11 0; 0 I]: a column
//     at position j < k solves R11 x = e_j (a column of R11^-1, for the row
//     norms 1/omega_i), a column at position >= k solves R11 n = R12 e_j (a
//     column of N);
//   * grid order is column order, so the canonical output (skeleton indices
//     ascending, then the rest) is one block scan of the skeleton counts.
// A swap relabels, rebuilds the columns from the basis and refactors the
// first k positions without pivoting, as k_compr does.
// ------------------------------------------------------------------------
template <int CMAX, int NT, int LPC, int J>
__global__ void __launch_bounds__(NT, 2) k_compr_w(IdArgs A) {
  constexpr int RL = CMAX / LPC;  // rows per lane and column
  constexpr int NC = NT / LPC * J;  // grid columns per workgroup
  constexpr int NW = NT / WAVE;   // wavefronts
  constexpr int VS = RL + 2;      // stride of a row phase in a column slot (phases on other banks)
  constexpr int SL = LPC * VS;    // one column slot
  constexpr int LDI = CMAX + 1;   // row stride of R11^-1
  // dynamic LDS, one region used in turn: the one-dimensional basis factors
  // [d*p][NC] while the basis is built; R11 by column j and row phase hh at
  // ((j*LPC + hh) * RL), zero on and below the diagonal; R11^-1 by rows
  extern __shared__ double dyn[];
  double *const Fl = dyn;
  double *const Rs = dyn;
  double *const Ris = dyn;
  __shared__ double xi[3 * ID_PMAX], wk[ID_PMAX], chc[ID_PMAX];
  __shared__ double pv[2 * NW * SL], rdiag[CMAX], rdg[CMAX], rinv[CMAX];
  __shared__ int srank[CMAX];
  __shared__ ArgMax ared[NW + 1], ared2[2 * NW];
  __shared__ int64_t sred[NT / WAVE + 1];
  const int tid = threadIdx.x;
  const int cb = tid / LPC, h = tid % LPC;  // column group, row phase
  const int wid = tid / WAVE, lane = tid & (WAVE - 1);
  const int p = A.p, d = A.d;
  if (tid < p) {
    double th = M_PI * (2.0 * tid + 1.0) / (2.0 * p);
    chc[tid] = cos(th);
    wk[tid] = ((tid & 1) ? -1.0 : 1.0) * sin(th);
  }
  const int e0 = A.order ? *A.ord_lo : 0;
  for (int e = e0 + blockIdx.x; e < A.ne - A.nb; e += gridDim.x) {
    const int i = A.order ? A.order[e] : A.nb + e;
    const int m = A.m[i];
    const int ks = A.S ? A.ks[i] : 0;
    const int c = A.c0 + ks;
    __syncthreads();
    if (tid < d * p) {
      int t = tid / p, q = tid % p;
      double lo = A.lo[3 * i + t], hi = A.hi[3 * i + t];
      xi[t * ID_PMAX + q] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * chc[q];
    }
    __syncthreads();
    if (m == 0) {
      if (tid == 0) A.k_out[i] = 0;
      continue;
    }
    bool act[J];
    int pa[J];  // current position of each column
    double col[J][RL], nrm[J];
#pragma unroll
    for (int j = 0; j < J; j++) {
      act[j] = J * cb + j < m;
      pa[j] = J * cb + j;
      nrm[j] = -1.0;
    }

    // the columns of C^T from the basis (barycentric tensor Lagrange values,
    // then the near-field vector entries), and their norms.  The group
    // shares the one-dimensional factors: phase h computes nodes q = h
    // (mod LPC).
    auto build_column = [&]() {
#pragma unroll
      for (int j = 0; j < J; j++) {
        if (!act[j]) continue;
        const int a = J * cb + j;
        const int64_t id = A.slot_id[A.gbeg[i] + a];
        for (int t = 0; t < d; t++) {
          const double x = A.P[id * d + t];
          const double lo = A.lo[3 * i + t], hi = A.hi[3 * i + t];
          double *Ft = Fl + (t * p) * NC + a;
          if (A.taylor_g > 0.0) {  // (uniform over the workgroup)
            for (int q = h; q < p; q += LPC)
              Ft[q * NC] = hi - lo == 0.0 ? (q == 0 ? 1.0 : 0.0) : taylor_phi(x, lo, hi, q, A.taylor_g);
            continue;
          }
          int hit = -1;
          double den = 0.0;
          if (hi - lo == 0.0) {
            hit = 0;
          } else {
            for (int q = h; q < p; q += LPC) {
              const double xq = xi[t * ID_PMAX + q];
              if (x == xq) {
                hit = q;
                break;
              }
              const double w = wk[q] / (x - xq);
              Ft[q * NC] = w;
              den += w;
            }
          }
          hit = group_max<LPC>(hit);
          den = group_sum<LPC>(den);
          if (hit >= 0)
            for (int q = h; q < p; q += LPC) Ft[q * NC] = q == hit ? 1.0 : 0.0;
          else
            for (int q = h; q < p; q += LPC) Ft[q * NC] = Ft[q * NC] / den;
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < J; j++) {
        if (act[j]) {
          const int a = J * cb + j;
          // row r = (k0 p + k1) p + k2 of the basis, r = LPC u + h
          int k2 = h % p, k1 = (h / p) % p, k0 = h / (p * p);
          const double *Sa = ks > 0 ? A.S + A.S_off[i - A.nb] + (int64_t)a * ks : nullptr;
#pragma unroll
          for (int u = 0; u < RL; u++) {
            const int r = LPC * u + h;
            double val = 0.0;
            if (r < A.c0) {
              if (d == 1)
                val = Fl[k2 * NC + a];
              else if (d == 2)
                val = Fl[(p + k2) * NC + a] * Fl[k1 * NC + a];
              else
                val = Fl[(2 * p + k2) * NC + a] * Fl[(p + k1) * NC + a] * Fl[k0 * NC + a];
              if (A.dlw)
                val = val * A.pdat[3 * (int64_t)A.slot_id[A.gbeg[i] + a] + (r < A.pd ? 0 : 1)];
            } else if (r < c) {
              val = Sa[r - A.c0];
            }
            col[j][u] = val;
            k2 += LPC;
            while (k2 >= p) {
              k2 -= p;
              if (++k1 == p) {
                k1 = 0;
                ++k0;
              }
            }
          }
          double s0 = 0.0;
#pragma unroll
          for (int u = 0; u < RL; u++) s0 = fma(col[j][u], col[j][u], s0);
          nrm[j] = group_sum<LPC>(s0);  // squared: the arg-max needs no root
        } else {
#pragma unroll
          for (int u = 0; u < RL; u++) col[j][u] = 0.0;
        }
      }
      __syncthreads();  // the factors are read before LDS is reused
    };

    // Householder QR over positions 0..kend-1: with pivoting the pivot of
    // step t is the largest remaining norm and the loop stops at the rank
    // test (|R_tt| <= tol * |R_00|); without, the pivot is position t.
    // Steps run in blocks of eight rows (tb unrolled): rows below 8 tb are
    // final in every remaining column, so a step touches local rows from
    // 8 tb / LPC on and masks by the runtime step only inside its block.
    // The pivot column keeps its registers (rows < t are its column of R)
    // and R_tt goes to rdiag.
    auto householder_qr = [&](bool pivoting, int kend) -> int {
      int kk = 0;
      double r00 = 0.0;
      bool stop = kend <= 0;
#pragma unroll
      for (int tb = 0; tb < CMAX / 8; tb++) {
        if (stop) break;
        const int r0 = 8 * tb, u0 = r0 / LPC, u1 = u0 + 8 / LPC;
        for (int tt = 0; tt < 8; tt++) {
          const int t = r0 + tt;
          if (t >= kend) {
            stop = true;
            break;
          }
          // every lane of a group holds its group's candidate (norms and
          // positions are the same in the group's lanes)
          ArgMax am{-1.0, -1};
#pragma unroll
          for (int j = 0; j < J; j++)
            if (act[j] && (pivoting ? pa[j] >= t : pa[j] == t))
              am = amax_pick(am, ArgMax{nrm[j], pa[j]});
          // each wavefront's own winner copies its column into the wave's
          // slot before the one barrier of the step, so the pivot column is
          // in LDS as soon as the block arg-max is known.  Slots and arg-max
          // entries alternate by step parity: a half is rewritten two steps
          // after it was read, with the barrier of the step in between.
          static_assert(LPC == 4, "the quad arg-max needs groups of four lanes");
          const ArgMax wa = wave_argmax_quad(am);
          double *const slots = pv + (t & 1) * (NW * SL);
          ArgMax *const ah = ared2 + (t & 1) * NW;
#pragma unroll
          for (int j = 0; j < J; j++) {
            if (act[j] && pa[j] == wa.a) {
              double *vs = slots + wid * SL + h * VS;
#pragma unroll
              for (int u = u0; u < RL; u++) vs[u] = col[j][u];
            }
          }
          if (lane == 0) ah[wid] = wa;
          __syncthreads();
          const ArgMax we = lane < NW ? ah[lane] : ArgMax{-1.0, -1};
          am = lanes_argmax<NW>(we);
          const double bn = sqrt(am.v);  // the pivot norm (the winner's root only)
          if (pivoting) {
            if (t == 0) {
              r00 = bn;
              if (!(r00 > 0.0)) {
                stop = true;
                break;
              }
            } else if (!(bn > A.tol * r00)) {
              stop = true;
              break;
            }
          }
          const int bp = am.a;
          if (bp < 0) {  // no column left at this position (uniform)
            stop = true;
            break;
          }
          // the wavefront whose winner is the pivot (positions are distinct)
          const uint64_t wins = __ballot(lane < NW && we.a == bp);
          const int ws = (int)__ffsll((unsigned long long)wins) - 1;
#pragma unroll
          for (int j = 0; j < J; j++) {
            if (act[j]) {
              if (pa[j] == t)
                pa[j] = bp;
              else if (pa[j] == bp)
                pa[j] = t;
            }
          }
          // v: zero above row t, x_t - R_tt at row t, the column below;
          // v^T v = 2 beta (beta + |x_t|) with beta the pivot norm
          const double *const src = slots + ws * SL;
          const double xt = src[(t % LPC) * VS + t / LPC];
          const double rtt = xt >= 0.0 ? -bn : bn;
          const double vn = 2.0 * bn * (bn + fabs(xt));
          const double rv = 2.0 / vn;
          if (tid == 0) rdiag[t] = rtt;
          const double *vh = src + h * VS;
          auto vval = [&](int u) -> double {
            const double y = vh[u];
            if (u >= u1) return y;
            const int r = LPC * u + h;
            return r < t ? 0.0 : (r == t ? y - rtt : y);
          };
          // two partial sums per column (even and odd rows of the lane):
          // half the chain of dependent multiply-adds
          double w[2][J];
#pragma unroll
          for (int j = 0; j < J; j++) w[0][j] = w[1][j] = 0.0;
#pragma unroll
          for (int u = u0; u < RL; u++) {
            const double vu = vval(u);
#pragma unroll
            for (int j = 0; j < J; j++) w[u & 1][j] = fma(vu, col[j][u], w[u & 1][j]);
          }
          // scale 0 leaves a column as it is (the pivot, finished ones)
          double sc[J];
          bool up[J];
#pragma unroll
          for (int j = 0; j < J; j++) {
            up[j] = act[j] && pa[j] > t && vn > 0.0;
            const double g = group_sum<LPC>(w[0][j] + w[1][j]);
            sc[j] = up[j] ? g * rv : 0.0;
          }
          // v is read again from LDS below rather than kept in registers
          __asm__ volatile("" ::: "memory");
          double s[2][J];
#pragma unroll
          for (int j = 0; j < J; j++) s[0][j] = s[1][j] = 0.0;
#pragma unroll
          for (int u = u0; u < RL; u++) {
            const double vu = vval(u);
            const bool below = u >= u1 || LPC * u + h > t;
#pragma unroll
            for (int j = 0; j < J; j++) {
              const double y = fma(-sc[j], vu, col[j][u]);
              col[j][u] = y;
              const double z = below ? y : 0.0;
              s[u & 1][j] = fma(z, z, s[u & 1][j]);
            }
          }
#pragma unroll
          for (int j = 0; j < J; j++) {
            const double nn = group_sum<LPC>(s[0][j] + s[1][j]);
            if (up[j]) nrm[j] = nn;
          }
          kk = t + 1;
        }
      }
      __syncthreads();
      return kk;
    };

    build_column();
    int k = householder_qr(true, m < c ? m : c);
    const int nr = m - k;
    int nsw = 0;
    bool failed = false;
    int exj[J];  // skeleton columns before column j of the group
    for (;;) {
      // skeleton ranks: grid order is column order
      int cnt = 0;
#pragma unroll
      for (int j = 0; j < J; j++) {
        exj[j] = cnt;
        cnt += (act[j] && pa[j] < k) ? 1 : 0;
      }
      int64_t tot;
      const int ex0 =
          (int)block_excl_scan_i64<NT / WAVE>(h == 0 ? cnt : 0, &tot, sred) - (h > 0 ? cnt : 0);
#pragma unroll
      for (int j = 0; j < J; j++) {
        exj[j] += ex0;
        if (h == 0 && act[j] && pa[j] < k) srank[pa[j]] = exj[j];
      }
      if (k == 0 || nr == 0) break;
      // R11 padded to [R11 0; 0 I]: strictly upper part by column and row
      // phase, the reciprocal diagonal (1 past k) in rdg
      if (k < CMAX) {
        for (int e = tid; e < CMAX * CMAX; e += NT) Rs[e] = 0.0;
        __syncthreads();
      }
#pragma unroll
      for (int j = 0; j < J; j++) {
        if (act[j] && pa[j] < k) {
          double *Rc = Rs + (pa[j] * LPC + h) * RL;
#pragma unroll
          for (int u = 0; u < RL; u++) Rc[u] = LPC * u + h < pa[j] ? col[j][u] : 0.0;
        }
      }
      if (tid < CMAX) rdg[tid] = tid < k ? 1.0 / rdiag[tid] : 1.0;
      __syncthreads();
      // right-hand side e_j at positions j < k; R12 columns stay in place
#pragma unroll
      for (int j = 0; j < J; j++) {
        if (pa[j] < k) {
#pragma unroll
          for (int u = 0; u < RL; u++) col[j][u] = LPC * u + h == pa[j] ? 1.0 : 0.0;
        }
      }
      // back substitution by columns of R11 in every lane (rows >= k see
      // the identity and leave the solution unchanged)
#pragma unroll
      for (int jj = CMAX - 1; jj >= 0; jj--) {
        const int uj = jj / LPC, hj = jj % LPC;
        const double rj = rdg[jj];
        double x[J];
#pragma unroll
        for (int j = 0; j < J; j++) {
          double xv = col[j][uj] * rj;
          if constexpr (LPC == 4) {
            xv = hj == 0   ? group_bcast<4, 0>(xv)
                 : hj == 1 ? group_bcast<4, 1>(xv)
                 : hj == 2 ? group_bcast<4, 2>(xv)
                           : group_bcast<4, 3>(xv);
          } else if constexpr (LPC == 2) {
            xv = hj == 0 ? group_bcast<2, 0>(xv) : group_bcast<2, 1>(xv);
          }
          x[j] = xv;
          if (h == hj) col[j][uj] = xv;
        }
        const double *Rc = Rs + (jj * LPC + h) * RL;
#pragma unroll
        for (int u = 0; u <= uj; u++) {
          const double r = Rc[u];
#pragma unroll
          for (int j = 0; j < J; j++) col[j][u] = fma(-r, x[j], col[j][u]);
        }
      }
      __syncthreads();  // every read of R11 is done before R11^-1 overwrites it
#pragma unroll
      for (int j = 0; j < J; j++) {
        if (act[j] && pa[j] < k) {
#pragma unroll
          for (int u = 0; u < RL; u++) Ris[(LPC * u + h) * LDI + pa[j]] = col[j][u];
        }
      }
      __syncthreads();
      // row norms of R11^-1
      if (tid < k) {
        double sq = 0.0;
        for (int jc = 0; jc < k; jc++) {
          const double y = Ris[tid * LDI + jc];
          sq = fma(y, y, sq);
        }
        rinv[tid] = sqrt(sq);
      }
      __syncthreads();
      // rho_ij^2 = N_ij^2 + (gamma_j / omega_i)^2; arg-max, ties: smallest
      // j, then smallest i (pair index j*k + i).  G rows are written on
      // every pass; the last pass leaves the final ones.  With gt_out the
      // lanes write G^T: for each skeleton index the rows of consecutive
      // columns are consecutive in memory.
      ArgMax am{-1.0, -1};
#pragma unroll
      for (int j = 0; j < J; j++) {
        if (act[j] && pa[j] >= k) {
          const double gam = sqrt(nrm[j]);  // norm of the column's rows >= k
          const int64_t row = J * cb + j - exj[j];
          double *Gr = A.G_out + A.go[i] + (A.gt_out ? row : row * k);
          const int64_t cs = A.gt_out ? (int64_t)nr : 1;
          // the other orientation as well (no transposition pass after)
          double *G2 = A.G2_out ? A.G2_out + A.go[i] + (A.gt_out ? row * k : row) : nullptr;
          const int64_t cs2 = A.gt_out ? 1 : (int64_t)nr;
          const int base = (pa[j] - k) * k;
#pragma unroll
          for (int u = 0; u < RL; u++) {
            const int ii = LPC * u + h;
            if (ii < k) {
              const double gw = gam * rinv[ii];
              const double r2 = col[j][u] * col[j][u] + gw * gw;
              am = amax_pick(am, ArgMax{r2, base + ii});
              Gr[srank[ii] * cs] = col[j][u];
              if (G2) G2[srank[ii] * cs2] = col[j][u];
            }
          }
        }
      }
      am = block_argmax<NT / WAVE>(am, ared);
      if (!(sqrt(am.v) > A.f)) break;
      if (++nsw > 64 * k) {
        failed = true;
        break;
      }
      const int bj = am.a / k, bi = am.a % k;
#pragma unroll
      for (int j = 0; j < J; j++) {
        if (act[j]) {
          if (pa[j] == bi)
            pa[j] = k + bj;
          else if (pa[j] == k + bj)
            pa[j] = bi;
        }
      }
      __syncthreads();  // R11^-1 reads are done before the factors reuse LDS
      build_column();
      householder_qr(false, k);
    }
    if (tid == 0 && nsw > 0) atomicAdd(A.swaps, nsw);
    // canonical output: skeleton indices ascending, then the rest
    if (h == 0) {
      int *sel = A.sel_out + A.selo[i];
#pragma unroll
      for (int j = 0; j < J; j++) {
        if (act[j]) {
          const int a = J * cb + j;
          if (failed)
            sel[a] = a;
          else if (pa[j] < k)
            sel[exj[j]] = a;
          else
            sel[k + (a - exj[j])] = a;
        }
      }
    }
    if (failed) {
      if (tid == 0) atomicOr(A.err, 1);
      k = 0;
    }
    if (tid == 0) A.k_out[i] = k;
  }
}

// ------------------------------------------------------------------------
// compr for wide bases and large grids (beyond the register form's c <= 64
// and m <= 256).  The algorithm and its conventions are those of k_compr_w:
// positions are labels (a pivot or a Gu-Eisenstat swap relabels two
// columns), the pivot is the largest squared residual norm with ties to the
// lowest position, each Householder step has one barrier (every wavefront
// stages its candidate column in LDS before it), the swap test solves R11
// by column back substitution with the reciprocal diagonal, and the
// canonical output comes from a block scan.  What differs is where the
// columns of M = C^T live: in a column-major tile (column a at a * ldc,
// rows contiguous) that every step streams through registers once -- in
// LDS when the node's tile fits there, else in a per-workgroup global
// scratch that stays in L2 and the infinity cache.  Groups of 16 lanes own
// columns a = g, g + 32, ... (lane h holds rows h, h + 16, ...), so a
// column slice is one 128-byte segment per 16 rows and a column sum is four
// DPP exchanges inside the group.  A launch takes its nodes from a list
// ordered by decreasing grid size, so the longest nodes start first.
constexpr int CS_NT = 512;
constexpr int CS_LPC = 16;
constexpr int CS_NG = CS_NT / CS_LPC;  // column groups
constexpr int CS_NW = CS_NT / WAVE;    // wavefronts

struct CsArgs {
  const int *order;  // node ids of the level, largest grid first
  const int *cnt;    // device: the launch takes order[0, *cnt)
  int ldc;           // column stride of the tile (a multiple of 16, >= c)
  int lds_cols;      // grids of at most this many points keep the tile in LDS
  int mmax;          // largest grid of the level
  double *gscr;      // per workgroup: tile (mmax x ldc), norms (mmax), R11^-1 (CMAX^2)
  int64_t gstride;
  int *iscr;         // per workgroup: labels (mmax), skeleton counts (mmax)
  int64_t istride;
  const int *first;  // device: the launch takes order[*first, *cnt) (null: from 0)
};

// the same inside a group of 8 lanes (a DPP half row)
__device__ __forceinline__ double g8_sum(double x) {
  x += perm_f64<0xB1>(x);   // quad_perm [1,0,3,2]
  x += perm_f64<0x4E>(x);   // quad_perm [2,3,0,1]
  x += perm_f64<0x141>(x);  // row_half_mirror: the other quad of the half row
  return x;
}

// sums, maxima and broadcasts inside a group of 16 lanes (one DPP row);
// every lane of the group ends with the same bits
__device__ __forceinline__ double g16_sum(double x) {
  x += perm_f64<0xB1>(x);   // quad_perm [1,0,3,2]
  x += perm_f64<0x4E>(x);   // quad_perm [2,3,0,1]
  x += perm_f64<0x141>(x);  // row_half_mirror: the other quad of the half row
  x += perm_f64<0x140>(x);  // row_mirror: the other half of the row
  return x;
}
__device__ __forceinline__ int g16_max(int x) {
  x = max(x, perm_i32<0xB1>(x));
  x = max(x, perm_i32<0x4E>(x));
  x = max(x, perm_i32<0x141>(x));
  x = max(x, perm_i32<0x140>(x));
  return x;
}

struct CsShared {
  const double *xi, *wk;
  double *slots, *Fg, *rdiag, *rdg, *rinv;
  int *piv, *msrc;
  ArgMax *meta, *ared;
  int64_t *sred;
};

// One node: W (tile), nrm2 (squared residual norms), lab (position labels),
// exs (skeleton columns before each grid index) in LDS (LT) or in the
// workgroup's global scratch; Rinv (R11^-1, k x k by columns) global; Lr
// (global tile only) LDS for rcap columns of R11 at a time.
template <int CMAX, bool LT>
__device__ __forceinline__ void compr_node_s(const IdArgs &A, const CsArgs &B, int i, int m,
                                             double *W, double *nrm2, int *lab, int *exs,
                                             double *Rinv, double *Lr, int rcap,
                                             const CsShared &sh) {
  constexpr int RL = CMAX / CS_LPC;    // rows per lane
  constexpr int JB = RL <= 8 ? 4 : 2;  // columns per pass of a group (QR)
  constexpr int JT = RL <= 8 ? 4 : RL <= 16 ? 2 : 1;  // (the back substitution)
  const int tid = threadIdx.x, g = tid / CS_LPC, h = tid % CS_LPC;
  const int wid = tid / WAVE, lane = tid & (WAVE - 1);
  const int ks = A.S ? A.ks[i] : 0;
  const int c = A.c0 + ks;
  const int ldc = B.ldc;
  const int d = A.d, p = A.p;

  // the columns of C^T from the basis (barycentric tensor Lagrange values,
  // then the near-field vector entries) and their squared norms; labels
  // start as the grid index unless `keep` (a refactorization after a swap)
  auto build = [&](bool keep) {
    for (int a0 = 0; a0 < m; a0 += CS_NG) {
      const int a = a0 + g;
      const bool on = a < m;
      double *F = sh.Fg + g * (d * p);
      if (on) {
        const int64_t id = A.slot_id[A.gbeg[i] + a];
        for (int t = 0; t < d; t++) {
          const double x = A.P[id * d + t];
          const double lo = A.lo[3 * i + t], hi = A.hi[3 * i + t];
          if (A.taylor_g > 0.0) {  // (uniform over the workgroup)
            for (int q = h; q < p; q += CS_LPC)
              F[t * p + q] = hi - lo == 0.0 ? (q == 0 ? 1.0 : 0.0) : taylor_phi(x, lo, hi, q, A.taylor_g);
            continue;
          }
          int hit = -1;
          double den = 0.0;
          if (hi - lo == 0.0) {
            hit = 0;
          } else {
            for (int q = h; q < p; q += CS_LPC) {
              const double xq = sh.xi[t * ID_PMAX + q];
              if (x == xq) {
                hit = q;
                break;
              }
              const double w = sh.wk[q] / (x - xq);
              F[t * p + q] = w;
              den += w;
            }
          }
          hit = g16_max(hit);
          den = g16_sum(den);
          for (int q = h; q < p; q += CS_LPC)
            F[t * p + q] = hit >= 0 ? (q == hit ? 1.0 : 0.0) : F[t * p + q] / den;
        }
      }
      __syncthreads();
      if (on) {
        const double *Sa = ks > 0 ? A.S + A.S_off[i - A.nb] + (int64_t)a * ks : nullptr;
        double s2 = 0.0;
#pragma unroll
        for (int u = 0; u < RL; u++) {
          const int r = CS_LPC * u + h;
          if (r < c) {
            double val;
            if (r < A.c0) {
              int q = r;
              val = 1.0;
              for (int t = d - 1; t >= 0; t--) {
                val *= F[t * p + q % p];
                q /= p;
              }
              if (A.dlw)
                val = val * A.pdat[3 * (int64_t)A.slot_id[A.gbeg[i] + a] + (r < A.pd ? 0 : 1)];
            } else {
              val = Sa[r - A.c0];
            }
            W[(int64_t)a * ldc + r] = val;
            s2 = fma(val, val, s2);
          }
        }
        s2 = g16_sum(s2);
        if (h == 0) {
          nrm2[a] = s2;
          if (!keep) lab[a] = a;
        }
      }
      __syncthreads();
    }
  };

  // Each wavefront's candidate for step t: the group holding the wave's
  // arg-max copies its column into the wave's slot.  Every lane copies the
  // rows it wrote itself in the last update (so it reads its own stores).
  // Slots and entries alternate by step parity.
  auto stage = [&](int t, ArgMax best, int bst) {
    const ArgMax wa = wave_argmax(best);
    const int e = (t & 1) * CS_NW + wid;
    if (wa.a >= 0 && best.a == wa.a) {
      double *slot = sh.slots + (int64_t)e * ldc;
      const double *cp = W + (int64_t)bst * ldc;
#pragma unroll
      for (int u = 0; u < RL; u++) {
        const int r = CS_LPC * u + h;
        if (r >= t && r < c) slot[r] = cp[r];
      }
      if (h == 0) {
        sh.meta[e] = wa;
        sh.msrc[e] = bst;
      }
    }
    if (wa.a < 0 && lane == 0) {
      sh.meta[e] = ArgMax{-1.0, -1};
      sh.msrc[e] = -1;
    }
  };

  // Householder QR over positions 0..kend-1: with pivoting the pivot of
  // step t is the largest remaining norm and the loop stops at the rank
  // test (|R_tt| <= tol |R_00|); without, it is the column labelled t.
  // Rows < t of a column are its column of R and stay in place; R_tt goes
  // to rdiag and the storage index of position t to piv.
  auto qr = [&](bool pivoting, int kend) -> int {
    if (kend <= 0) return 0;
    {
      ArgMax best{-1.0, -1};
      int bst = -1;
      for (int a = g; a < m; a += CS_NG) {
        const int la = lab[a];
        if (pivoting || la == 0) {
          const ArgMax y = amax_pick(best, ArgMax{nrm2[a], la});
          if (y.a == la && best.a != la) {
            best = y;
            bst = a;
          }
        }
      }
      stage(0, best, bst);
    }
    int kk = 0;
    double r00 = 0.0;
    for (int t = 0; t < kend; t++) {
      __syncthreads();
      const int e0 = (t & 1) * CS_NW;
      const ArgMax we = lane < CS_NW ? sh.meta[e0 + lane] : ArgMax{-1.0, -1};
      const ArgMax am = lanes_argmax<CS_NW>(we);
      const double bn = sqrt(am.v);
      if (pivoting) {
        if (t == 0) {
          r00 = bn;
          if (!(r00 > 0.0)) break;
        } else if (!(bn > A.tol * r00)) {
          break;
        }
      }
      const int bp = am.a;
      if (bp < 0) break;
      const uint64_t wins = __ballot(lane < CS_NW && we.a == bp);
      const int ws = (int)__ffsll((unsigned long long)wins) - 1;
      const int b = sh.msrc[e0 + ws];
      const double *src = sh.slots + (int64_t)(e0 + ws) * ldc;
      const double xt = src[t];
      const double rtt = xt >= 0.0 ? -bn : bn;
      const double vn = 2.0 * bn * (bn + fabs(xt));
      const double rv = 2.0 / vn;
      if (tid == 0) {
        sh.rdiag[t] = rtt;
        sh.piv[t] = b;
      }
      // v: zero above row t, x_t - R_tt at row t, the column below
      double v[RL];
#pragma unroll
      for (int u = 0; u < RL; u++) {
        const int r = CS_LPC * u + h;
        v[u] = (r < t || r >= c) ? 0.0 : (r == t ? src[r] - rtt : src[r]);
      }
      ArgMax best{-1.0, -1};
      int bst = -1;
      // JB columns per pass of the group: their loads are in flight together
      for (int a0 = g; a0 < m; a0 += CS_NG * JB) {
        int na[JB];
        bool on[JB];
        double col[JB][RL];
#pragma unroll
        for (int j = 0; j < JB; j++) {
          const int a = a0 + CS_NG * j;
          on[j] = a < m;
          const int la = on[j] ? lab[a] : -1;
          na[j] = a == b ? t : (la == t ? bp : la);  // positions t and bp swap
          if (on[j] && na[j] != la && h == 0) lab[a] = na[j];
          on[j] = on[j] && na[j] > t;  // not the pivot of this step or an earlier one
          const double *cp = W + (int64_t)a * ldc;
#pragma unroll
          for (int u = 0; u < RL; u++) {
            const int r = CS_LPC * u + h;
            col[j][u] = (on[j] && r >= t && r < c) ? cp[r] : 0.0;
          }
        }
        // two partial sums per column: half the chain of dependent multiply-adds
        double sc[JB];
#pragma unroll
        for (int j = 0; j < JB; j++) {
          double w0 = 0.0, w1 = 0.0;
#pragma unroll
          for (int u = 0; u < RL; u += 2) {
            w0 = fma(v[u], col[j][u], w0);
            if (u + 1 < RL) w1 = fma(v[u + 1], col[j][u + 1], w1);
          }
          sc[j] = g16_sum(w0 + w1);
        }
#pragma unroll
        for (int j = 0; j < JB; j++) {
          const double scj = (on[j] && vn > 0.0) ? sc[j] * rv : 0.0;
          double *cp = W + (int64_t)(a0 + CS_NG * j) * ldc;
          double s0 = 0.0, s1 = 0.0;
#pragma unroll
          for (int u = 0; u < RL; u++) {
            const int r = CS_LPC * u + h;
            const double y = fma(-scj, v[u], col[j][u]);
            col[j][u] = y;
            if (on[j] && r >= t && r < c) cp[r] = y;
            const double z = r > t ? y : 0.0;
            if (u & 1)
              s1 = fma(z, z, s1);
            else
              s0 = fma(z, z, s0);
          }
          sc[j] = s0 + s1;
        }
#pragma unroll
        for (int j = 0; j < JB; j++) {
          const double nn = g16_sum(sc[j]);
          if (!on[j]) continue;
          if (h == 0) nrm2[a0 + CS_NG * j] = nn;
          if (pivoting || na[j] == t + 1) {
            const ArgMax y = amax_pick(best, ArgMax{nn, na[j]});
            if (y.a == na[j] && best.a != na[j]) {
              best = y;
              bst = a0 + CS_NG * j;
            }
          }
        }
      }
      kk = t + 1;
      if (t + 1 < kend) stage(t + 1, best, bst);
    }
    __syncthreads();
    return kk;
  };

  build(false);
  int k = qr(true, m < c ? m : c);
  const int nr = m - k;
  int nsw = 0;
  bool failed = false;
  for (;;) {
    // skeleton columns before each grid index (grid order is storage order)
    {
      const int chunk = (m + CS_NT - 1) / CS_NT;
      const int a0 = tid * chunk;
      int cnt = 0;
      for (int e = 0; e < chunk && a0 + e < m; e++) cnt += lab[a0 + e] < k ? 1 : 0;
      int64_t tot;
      int ex = (int)block_excl_scan_i64<CS_NW>(cnt, &tot, sh.sred);
      for (int e = 0; e < chunk && a0 + e < m; e++) {
        exs[a0 + e] = ex;
        ex += lab[a0 + e] < k ? 1 : 0;
      }
      __syncthreads();
    }
    if (k == 0 || nr == 0) break;
    if (tid < k) sh.rdg[tid] = 1.0 / sh.rdiag[tid];
    __syncthreads();
    // back substitution by columns of R11 (column j: rows < j of the tile
    // column piv[j], diagonal rdiag[j]) in every column: a column at
    // position j < k solves R11 x = e_j (a column of R11^-1, kept in Rinv),
    // one at a position >= k solves R11 n = R12 e (a column of N, kept over
    // its rows < k; R11's columns are never overwritten).  With the tile in
    // LDS in one pass; otherwise R11 passes through LDS (Lr, rcols columns
    // at a time, last columns first) and the vectors are reloaded per pass.
    for (int a = g; a < m; a += CS_NG) {
      const int la = lab[a];
      if (la < k) {
#pragma unroll
        for (int u = 0; u < RL; u++) {
          const int r = CS_LPC * u + h;
          if (r < k) Rinv[(int64_t)la * k + r] = r == la ? 1.0 : 0.0;
        }
      }
    }
    const int rcols = LT ? k : rcap;
    for (int j1 = k; j1 > 0; j1 -= rcols) {
      const int j0 = j1 - rcols > 0 ? j1 - rcols : 0;
      __syncthreads();
      if constexpr (!LT) {
        for (int e = tid; e < (j1 - j0) * ldc; e += CS_NT) {
          const int jc = e / ldc, r = e - jc * ldc;
          if (r < j0 + jc) Lr[e] = W[(int64_t)sh.piv[j0 + jc] * ldc + r];
        }
        __syncthreads();
      }
      for (int a0 = g; a0 < m; a0 += CS_NG * JT) {
        double *xp[JT];
        double x[JT][RL];
#pragma unroll
        for (int j = 0; j < JT; j++) {
          const int a = a0 + CS_NG * j;
          const int la = a < m ? lab[a] : k;
          xp[j] = a >= m ? nullptr : la >= k ? W + (int64_t)a * ldc : Rinv + (int64_t)la * k;
#pragma unroll
          for (int u = 0; u < RL; u++) {
            const int r = CS_LPC * u + h;
            x[j][u] = (xp[j] && r < j1) ? xp[j][r] : 0.0;
          }
        }
        // blocks of 16 rows unrolled (register indices stay static), the
        // rows of a block in a loop
#pragma unroll
        for (int ub = RL - 1; ub >= 0; ub--) {
          const int jlo = CS_LPC * ub > j0 ? CS_LPC * ub : j0;
          const int jhi = CS_LPC * ub + CS_LPC < j1 ? CS_LPC * ub + CS_LPC : j1;
          if (jlo >= jhi) continue;
#pragma unroll 1
          for (int jj = jhi - 1; jj >= jlo; jj--) {
            const int hj = jj - CS_LPC * ub;
            const double rd = sh.rdg[jj];
            double xv[JT];
#pragma unroll
            for (int j = 0; j < JT; j++) {
              xv[j] = __shfl(x[j][ub], (lane & ~(CS_LPC - 1)) + hj, WAVE) * rd;
              if (h == hj) x[j][ub] = xv[j];
            }
            const double *Rc = LT ? W + (int64_t)sh.piv[jj] * ldc : Lr + (int64_t)(jj - j0) * ldc;
#pragma unroll
            for (int u = 0; u <= ub; u++) {
              const int r = CS_LPC * u + h;
              if (r < jj) {
                const double rr = Rc[r];
#pragma unroll
                for (int j = 0; j < JT; j++) x[j][u] = fma(-rr, xv[j], x[j][u]);
              }
            }
          }
        }
#pragma unroll
        for (int j = 0; j < JT; j++) {
          if (!xp[j]) continue;
#pragma unroll
          for (int u = 0; u < RL; u++) {
            const int r = CS_LPC * u + h;
            if (r < j1) xp[j][r] = x[j][u];
          }
        }
      }
    }
    __syncthreads();
    // row norms of R11^-1: a group per row, lane h summing the columns
    // jc = h (mod 16), then the group sum
    for (int ii = g; ii < k; ii += CS_NG) {
      double sq = 0.0;
      for (int jc = h; jc < k; jc += CS_LPC) {
        const double y = Rinv[(int64_t)jc * k + ii];
        sq = fma(y, y, sq);
      }
      sq = g16_sum(sq);
      if (h == 0) sh.rinv[ii] = sqrt(sq);
    }
    __syncthreads();
    // rho_ij^2 = N_ij^2 + (gamma_j / omega_i)^2; arg-max, ties: smallest j,
    // then smallest i (pair index j*k + i).  G rows are written on every
    // pass; the last pass leaves the final ones.
    ArgMax am{-1.0, -1};
    for (int a = g; a < m; a += CS_NG) {
      const int la = lab[a];
      if (la < k) continue;
      const double gam = sqrt(nrm2[a]);  // norm of the column's rows >= k
      double *Gr = A.G_out + A.go[i] + (int64_t)(a - exs[a]) * k;
      const int base = (la - k) * k;
      const double *cp = W + (int64_t)a * ldc;
#pragma unroll
      for (int u = 0; u < RL; u++) {
        const int ii = CS_LPC * u + h;
        if (ii < k) {
          const double nv = cp[ii];
          const double gw = gam * sh.rinv[ii];
          const double r2 = nv * nv + gw * gw;
          am = amax_pick(am, ArgMax{r2, base + ii});
          Gr[exs[sh.piv[ii]]] = nv;
        }
      }
    }
    am = block_argmax<CS_NW>(am, sh.ared);
    if (!(sqrt(am.v) > A.f)) break;
    if (++nsw > 64 * k) {
      failed = true;
      break;
    }
    const int bj = am.a / k, bi = am.a % k;
    for (int a = tid; a < m; a += CS_NT) {
      const int la = lab[a];
      if (la == bi)
        lab[a] = k + bj;
      else if (la == k + bj)
        lab[a] = bi;
    }
    __syncthreads();
    build(true);
    qr(false, k);
  }
  if (tid == 0 && nsw > 0) atomicAdd(A.swaps, nsw);
  // canonical output: skeleton indices ascending, then the rest
  int *sel = A.sel_out + A.selo[i];
  for (int a = tid; a < m; a += CS_NT) {
    if (failed) {
      sel[a] = a;
    } else {
      const int ex = exs[a];
      if (lab[a] < k)
        sel[ex] = a;
      else
        sel[k + (a - ex)] = a;
    }
  }
  if (failed) {
    if (tid == 0) atomicOr(A.err, 1);
    k = 0;
  }
  if (tid == 0) A.k_out[i] = k;
}

template <int CMAX>
__global__ void __launch_bounds__(CS_NT) k_compr_s(IdArgs A, CsArgs B) {
  extern __shared__ double dyn[];
  __shared__ double xi[3 * ID_PMAX], wk[ID_PMAX], chc[ID_PMAX];
  __shared__ double rdiag[CMAX], rdg[CMAX], rinv[CMAX];
  __shared__ int piv[CMAX], msrc[2 * CS_NW];
  __shared__ ArgMax meta[2 * CS_NW], ared[CS_NW + 1];
  __shared__ int64_t sred[CS_NW + 1];
  const int tid = threadIdx.x;
  const int p = A.p, d = A.d, ldc = B.ldc;
  if (tid < p) {
    const double th = M_PI * (2.0 * tid + 1.0) / (2.0 * p);
    chc[tid] = cos(th);
    wk[tid] = ((tid & 1) ? -1.0 : 1.0) * sin(th);
  }
  // dynamic LDS: the staging slots, the groups' one-dimensional factors,
  // then the LDS tile with its norms, labels and counts
  double *const slots = dyn;
  double *const Fg = slots + 2 * CS_NW * ldc;
  double *const Lw = Fg + CS_NG * d * p;
  double *const Ln = Lw + (int64_t)B.lds_cols * ldc;
  int *const Ll = (int *)(Ln + B.lds_cols);
  int *const Le = Ll + B.lds_cols;
  // the workgroup's global scratch
  double *const Gw = B.gscr + (int64_t)blockIdx.x * B.gstride;
  double *const Gn = Gw + (int64_t)B.mmax * ldc;
  double *const Ri = Gn + B.mmax;
  int *const Gl = B.iscr + (int64_t)blockIdx.x * B.istride;
  int *const Ge = Gl + B.mmax;
  const CsShared sh{xi, wk, slots, Fg, rdiag, rdg, rinv, piv, msrc, meta, ared, sred};
  const int cnt = *B.cnt;
  const int e0 = B.first ? *B.first : 0;
  for (int e = e0 + blockIdx.x; e < cnt; e += gridDim.x) {
    const int i = B.order ? B.order[e] : A.nb + e;
    const int m = A.m[i];
    __syncthreads();
    if (tid < d * p) {
      const int t = tid / p, q = tid % p;
      const double lo = A.lo[3 * i + t], hi = A.hi[3 * i + t];
      xi[t * ID_PMAX + q] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * chc[q];
    }
    __syncthreads();
    if (m == 0) {
      if (tid == 0) A.k_out[i] = 0;
      continue;
    }
    if (m <= B.lds_cols)
      compr_node_s<CMAX, true>(A, B, i, m, Lw, Ln, Ll, Le, Ri, nullptr, 0, sh);
    else  // the LDS tile area takes columns of R11 in the back substitution
      compr_node_s<CMAX, false>(A, B, i, m, Gw, Gn, Gl, Ge, Ri, Lw,
                                (int)(((int64_t)B.lds_cols * (ldc + 2)) / ldc), sh);
  }
}

// ------------------------------------------------------------------------
// compr with every grid column held in registers for the whole algorithm, a
// node's columns split over nw workgroups (nw = 1, 2, 4, 8 or 16 by grid
// size; DQ_CPW columns per workgroup, the grid range [w DQ_CPW, (w+1)
// DQ_CPW) in workgroup w).  The algorithm and its arithmetic are the wide
// form's above -- labels for positions, the pivot as the largest squared
// residual norm with ties to the lowest position, the reflector from the
// pivot norm, norms recomputed exactly in the update, the rank test
// against tol |R_00|; the swap test by column back substitution against
// R11 with the reciprocal diagonal, rho^2 = N_ij^2 + (gamma_j / omega_i)^2
// with its arg-max over pair indices, a swap relabelling two columns and
// refactoring from the rebuilt basis without pivoting; the canonical
// output -- in the same order of summation.  With nw > 1 the workgroups of
// a node meet where a step needs all of them: each publishes what it holds
// (its best column and candidate, its columns of R11 and R11^-1, its
// skeleton count, its rho candidate) through device-coherent atomic
// accesses, and a counter per group of nw workgroups, incremented once a
// workgroup's accesses have completed, tells when all have.  A grid holds
// at most the workgroups the device keeps resident, the workgroups of a
// group sit on one XCD, consecutive in its dispatch order, and one grid runs
// at a time (launch_dq_chained); a wait longer than spin_limit ticks of the
// 100 MHz clock gives up with the error flag instead of hanging.
// ------------------------------------------------------------------------
constexpr int DQ_CPG = 4;               // columns per 16-lane group
constexpr int DQ_CPW = CS_NG * DQ_CPG;  // columns per workgroup
constexpr int DQ_MAXW = 16;             // workgroups per node, at most

// The workgroups of a group wait for each other, so each group must be
// resident as a whole.  A grid holds at most as many workgroups as the
// device keeps resident at once, a group's workgroups are consecutive in the
// dispatch order of one XCD, and workgroups are dispatched in order: only the
// last dispatched group can be partly resident, every group before it is
// whole and finishes, and its slots go to the rest.  That holds while no
// other grid of k_compr_dq occupies the device, which constructions on
// several streams would otherwise do; so every such launch of the process on
// a device waits for the previous one (an event recorded after each, waited
// on by the next launch's stream), whatever stream it comes from.  Other
// kernels on other streams only delay a group: they never wait for it.
struct LaunchChain {
  std::mutex mu;
  hipEvent_t last[64] = {};
};
static LaunchChain dq_chain;

// launches `kernel` on s after every earlier launch through this function on
// `device` (the caller's current device)
static void launch_dq_chained(int device, const void *kernel, int grid, int threads, void **args,
                              size_t shmem, hipStream_t s) {
  if (device < 0 || device >= 64) throw Error{SMASH_E_UNSUPPORTED, "device index above 63"};
  std::lock_guard<std::mutex> lock(dq_chain.mu);
  hipEvent_t &ev = dq_chain.last[device];
  if (!ev)
    SMASH_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  else
    SMASH_HIP(hipStreamWaitEvent(s, ev, 0));
  SMASH_HIP(hipLaunchKernel(kernel, dim3(grid), dim3(threads), args, shmem, s));
  SMASH_HIP(hipEventRecord(ev, s));
}

struct DqMeta {
  double v;  // candidate value (-1: none)
  int lab;   // its label (or pair index)
  int a;     // its storage (grid) index
};

struct DqArgs {
  const int *order;  // the level's wide-form nodes, largest grid first
  const int *range;  // device: positions [range[0], range[1]) of order for this launch
  int nw;            // workgroups per node
  int ldc;           // rows of an exchanged column (>= c)
  int *exs;          // per node at selo: skeleton columns before each grid index
  double *gslot;     // per group: [2][nw][ldc] published columns
  DqMeta *gmeta;     // per group: [3][nw] published candidates (QR steps by
                     // parity, the swap test)
  double *gR;        // per group: R11 by columns (k x k), then R11^-1 by columns
  double *gI;
  int gr_stride;     // entries of one group's gR / gI
  int *gcount;       // per group: [nw] skeleton counts
  unsigned *gcnt;    // per group: arrivals
  int64_t spin_limit;
};

template <int CMAX>
__global__ void __launch_bounds__(CS_NT) k_compr_dq(IdArgs A, DqArgs D) {
  extern __shared__ double dq_dyn[];  // the groups' one-dimensional factors, then R11 columns
  constexpr int RL = CMAX / CS_LPC;
  constexpr int RC = CMAX <= 224 ? 64 : 48;  // R11 columns staged in LDS at a time
  __shared__ double xi[3 * ID_PMAX], wk[ID_PMAX], chc[ID_PMAX];
  __shared__ double lslot[2][CS_NW][CMAX];
  __shared__ double rdiag[CMAX], rdg[CMAX], rinv[CMAX];
  __shared__ int piv[CMAX];
  __shared__ ArgMax wbest[2 * CS_NW];
  __shared__ int wsrc[2 * CS_NW];
  __shared__ ArgMax ared[CS_NW + 1];
  __shared__ int64_t sred[CS_NW + 1];
  __shared__ int sflag, sbase;
  const int tid = threadIdx.x, g = tid / CS_LPC, h = tid % CS_LPC;
  const int wid = tid / WAVE, lane = tid & (WAVE - 1);
  const int p = A.p, d = A.d, ldc = D.ldc, nw = D.nw;
  // the workgroups of a group on one XCD (workgroups go to the eight XCDs
  // round-robin), so their meetings stay within one L2
  const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8, gpx = gridDim.x / (8 * nw);
  const int grp = xcd * gpx + slot / nw, w = slot % nw, ngrp = 8 * gpx;
  if (tid < p) {
    const double th = M_PI * (2.0 * tid + 1.0) / (2.0 * p);
    chc[tid] = cos(th);
    wk[tid] = ((tid & 1) ? -1.0 : 1.0) * sin(th);
  }
  double *const F = dq_dyn + g * (d * p);
  double *const Lr = dq_dyn + CS_NG * d * p;  // RC columns of CMAX rows
  double *const gs = D.gslot + (int64_t)grp * 2 * nw * ldc;
  DqMeta *const gm = D.gmeta + (int64_t)grp * 3 * nw;
  double *const gR = D.gR + (int64_t)grp * D.gr_stride;
  double *const gI = D.gI + (int64_t)grp * D.gr_stride;
  int *const gc = D.gcount + (int64_t)grp * nw;
  unsigned nsync = 0;  // meetings of this group so far (the same in all its workgroups)
  bool abort = false;

  auto st = [&](double *q, double v) {
    __hip_atomic_store(q, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  auto ld = [&](const double *q) -> double {
    return __hip_atomic_load(const_cast<double *>(q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  auto sti = [&](int *q, int v) {
    __hip_atomic_store(q, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  auto ldi = [&](const int *q) -> int {
    return __hip_atomic_load(const_cast<int *>(q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  // all workgroups of the group have passed this point with their shared
  // writes complete (false: the wait timed out)
  auto meet = [&]() -> bool {
    if (nw == 1) {
      __syncthreads();
      return true;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    nsync++;
    if (tid == 0) {
      __hip_atomic_fetch_add(D.gcnt + grp, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned target = nsync * (unsigned)nw;
      const uint64_t t0 = wall_clock64();
      int to = 0;
      while (__hip_atomic_load(D.gcnt + grp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
             target) {
        if ((int64_t)(wall_clock64() - t0) > D.spin_limit) {
          to = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      sflag = to;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (sflag) {
      if (tid == 0) atomicOr(A.err, 2);
      return false;
    }
    return true;
  };
  // the group's arg-max of one candidate per workgroup (value, label;
  // a = storage index), returned to every lane
  auto group_argmax = [&](ArgMax mine, int mine_a, int par, int *win_w, int *win_a) -> ArgMax {
    if (nw == 1) {
      *win_w = 0;
      *win_a = mine_a;
      return mine;
    }
    if (tid == 0) {
      DqMeta *me = gm + par * nw + w;
      st(&me->v, mine.v);
      sti(&me->lab, mine.a);
      sti(&me->a, mine_a);
    }
    if (!meet()) {
      abort = true;
      return ArgMax{-1.0, -1};
    }
    double mv = -1.0;
    int ml = -1, ma = -1;
    if (lane < nw) {
      DqMeta *mp = gm + par * nw + lane;
      mv = ld(&mp->v);
      ml = ldi(&mp->lab);
      ma = ldi(&mp->a);
    }
    const ArgMax r = lanes_argmax<DQ_MAXW>(ArgMax{mv, ml});
    const uint64_t gw = __ballot(lane < nw && r.a >= 0 && ml == r.a);
    const int ws = gw ? (int)__ffsll((unsigned long long)gw) - 1 : 0;
    *win_w = ws;
    *win_a = r.a >= 0 ? __builtin_amdgcn_readlane(ma, ws) : -1;
    return r;
  };

  const int lo = D.range[0], hi = D.range[1];
  for (int e = lo + grp; e < hi; e += ngrp) {
    const int i = D.order[e];
    const int m = A.m[i];
    __syncthreads();
    if (tid < d * p) {
      const int t = tid / p, q = tid % p;
      const double blo = A.lo[3 * i + t], bhi = A.hi[3 * i + t];
      xi[t * ID_PMAX + q] = 0.5 * (blo + bhi) + 0.5 * (bhi - blo) * chc[q];
    }
    __syncthreads();
    if (m == 0) {
      if (w == 0 && tid == 0) A.k_out[i] = 0;
      continue;
    }
    const int ks = A.S ? A.ks[i] : 0;
    const int c = A.c0 + ks;
    double col[DQ_CPG][RL];
    double nr[DQ_CPG];
    int lb[DQ_CPG];

    // the columns of C^T from the basis and their squared norms; labels
    // start as the grid index unless `keep`
    auto build = [&](bool keep) {
#pragma unroll
      for (int j = 0; j < DQ_CPG; j++) {
        const int a = w * DQ_CPW + g + CS_NG * j;
        const bool on = a < m;
        if (on) {
          const int64_t id = A.slot_id[A.gbeg[i] + a];
          for (int t = 0; t < d; t++) {
            const double x = A.P[id * d + t];
            const double blo = A.lo[3 * i + t], bhi = A.hi[3 * i + t];
            if (A.taylor_g > 0.0) {  // (uniform over the workgroup)
              for (int q = h; q < p; q += CS_LPC)
                F[t * p + q] = bhi - blo == 0.0 ? (q == 0 ? 1.0 : 0.0)
                                                : taylor_phi(x, blo, bhi, q, A.taylor_g);
              continue;
            }
            int hit = -1;
            double den = 0.0;
            if (bhi - blo == 0.0) {
              hit = 0;
            } else {
              for (int q = h; q < p; q += CS_LPC) {
                const double xq = xi[t * ID_PMAX + q];
                if (x == xq) {
                  hit = q;
                  break;
                }
                const double wq = wk[q] / (x - xq);
                F[t * p + q] = wq;
                den += wq;
              }
            }
            hit = g16_max(hit);
            den = g16_sum(den);
            for (int q = h; q < p; q += CS_LPC)
              F[t * p + q] = hit >= 0 ? (q == hit ? 1.0 : 0.0) : F[t * p + q] / den;
          }
        }
        __syncthreads();
        double s2 = 0.0;
        const double *Sa = (on && ks > 0) ? A.S + A.S_off[i - A.nb] + (int64_t)a * ks : nullptr;
#pragma unroll
        for (int u = 0; u < RL; u++) {
          const int r = CS_LPC * u + h;
          double val = 0.0;
          if (on && r < c) {
            if (r < A.c0) {
              int q = r;
              val = 1.0;
              for (int t = d - 1; t >= 0; t--) {
                val *= F[t * p + q % p];
                q /= p;
              }
              if (A.dlw)
                val = val * A.pdat[3 * (int64_t)A.slot_id[A.gbeg[i] + a] + (r < A.pd ? 0 : 1)];
            } else {
              val = Sa[r - A.c0];
            }
            s2 = fma(val, val, s2);
          }
          col[j][u] = val;
        }
        nr[j] = g16_sum(s2);
        if (!keep) lb[j] = on ? a : -1;
        __syncthreads();
      }
    };

    // Householder QR over positions 0..kend-1 (pivoting: the largest
    // remaining norm, stop at the rank test; else the column labelled t);
    // R_tt and the storage index of position t go to rdiag / piv (LDS)
    auto qr = [&](bool pivoting, int kend) -> int {
      ArgMax best{-1.0, -1};
      int bst = -1;
#pragma unroll
      for (int j = 0; j < DQ_CPG; j++) {
        if (lb[j] < 0 || !(pivoting || lb[j] == 0)) continue;
        const ArgMax y = amax_pick(best, ArgMax{nr[j], lb[j]});
        if (y.a == lb[j] && best.a != lb[j]) {
          best = y;
          bst = j;
        }
      }
      int kk = 0;
      double r00 = 0.0;
      for (int t = 0; t < kend; t++) {
        const int par = t & 1;
        {  // each wavefront stages its best column (rows t..) and candidate
          const ArgMax wa = wave_argmax(best);
          const int ew = par * CS_NW + wid;
          if (wa.a >= 0 && best.a == wa.a) {
#pragma unroll
            for (int j = 0; j < DQ_CPG; j++)
              if (j == bst) {
#pragma unroll
                for (int u = 0; u < RL; u++) {
                  const int r = CS_LPC * u + h;
                  if (r >= t && r < c) lslot[par][wid][r] = col[j][u];
                }
              }
            if (h == 0) {
              wbest[ew] = wa;
              wsrc[ew] = w * DQ_CPW + g + CS_NG * bst;
            }
          }
          if (wa.a < 0 && lane == 0) {
            wbest[ew] = ArgMax{-1.0, -1};
            wsrc[ew] = -1;
          }
        }
        __syncthreads();
        const ArgMax we = lane < CS_NW ? wbest[par * CS_NW + lane] : ArgMax{-1.0, -1};
        const ArgMax wb = lanes_argmax<CS_NW>(we);
        const uint64_t wins = __ballot(lane < CS_NW && wb.a >= 0 && we.a == wb.a);
        const int wsl = wins ? (int)__ffsll((unsigned long long)wins) - 1 : 0;
        const int wa_idx = wb.a >= 0 ? wsrc[par * CS_NW + wsl] : -1;
        const double *src = &lslot[par][wsl][0];
        if (nw > 1 && wb.a >= 0) {
          double *mys = gs + ((int64_t)par * nw + w) * ldc;
          for (int r = t + tid; r < c; r += CS_NT) st(mys + r, src[r]);
        }
        int ws = 0, b = -1;
        const ArgMax am = group_argmax(wb, wa_idx, par, &ws, &b);
        if (abort) return kk;
        const bool remote = nw > 1 && ws != w;
        if (remote) src = gs + ((int64_t)par * nw + ws) * ldc;
        const double bn = sqrt(am.v);
        if (pivoting) {
          if (t == 0) {
            r00 = bn;
            if (!(r00 > 0.0)) break;
          } else if (!(bn > A.tol * r00)) {
            break;
          }
        }
        const int bp = am.a;
        if (bp < 0) break;
        auto rd = [&](int r) -> double { return remote ? ld(src + r) : src[r]; };
        const double xt = rd(t);
        const double rtt = xt >= 0.0 ? -bn : bn;
        const double vn = 2.0 * bn * (bn + fabs(xt));
        const double rv = 2.0 / vn;
        if (tid == 0) {
          rdiag[t] = rtt;
          piv[t] = b;
        }
        double v[RL];
#pragma unroll
        for (int u = 0; u < RL; u++) {
          const int r = CS_LPC * u + h;
          v[u] = (r < t || r >= c) ? 0.0 : (r == t ? rd(r) - rtt : rd(r));
        }
        best = ArgMax{-1.0, -1};
        bst = -1;
#pragma unroll
        for (int j = 0; j < DQ_CPG; j++) {
          const int a = w * DQ_CPW + g + CS_NG * j;
          const int la = lb[j];
          const bool on0 = la >= 0;
          const int na = a == b ? t : (la == t ? bp : la);  // positions t and bp swap
          if (on0) lb[j] = na;
          const bool on = on0 && na > t;  // not the pivot of this step or an earlier one
          double w0 = 0.0, w1 = 0.0;
#pragma unroll
          for (int u = 0; u < RL; u += 2) {
            w0 = fma(v[u], col[j][u], w0);
            if (u + 1 < RL) w1 = fma(v[u + 1], col[j][u + 1], w1);
          }
          const double sc = g16_sum(w0 + w1);
          const double scj = (on && vn > 0.0) ? sc * rv : 0.0;
          double s0 = 0.0, s1 = 0.0;
#pragma unroll
          for (int u = 0; u < RL; u++) {
            const int r = CS_LPC * u + h;
            const double y = fma(-scj, v[u], col[j][u]);
            col[j][u] = y;
            const double z = r > t ? y : 0.0;
            if (u & 1)
              s1 = fma(z, z, s1);
            else
              s0 = fma(z, z, s0);
          }
          const double nn = g16_sum(s0 + s1);
          if (on) {
            nr[j] = nn;
            if (pivoting || na == t + 1) {
              const ArgMax y = amax_pick(best, ArgMax{nn, na});
              if (y.a == na && best.a != na) {
                best = y;
                bst = j;
              }
            }
          }
        }
        kk = t + 1;
      }
      __syncthreads();
      return kk;
    };

    build(false);
    int k = qr(true, m < c ? m : c);
    if (abort) break;
    const int nr_ = m - k;
    int nsw = 0;
    bool failed = false;
    int skel_before = 0;  // skeleton columns in the workgroups before this one
    for (;;) {
      // skeleton counts: this workgroup's, then the prefix over the group
      {
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < DQ_CPG; j++) cnt += (lb[j] >= 0 && lb[j] < k && h == 0) ? 1 : 0;
        int64_t tot;
        (void)block_excl_scan_i64<CS_NW>(cnt, &tot, sred);
        if (nw > 1) {
          if (tid == 0) sti(gc + w, (int)tot);
          if (!meet()) {
            abort = true;
            break;
          }
          if (tid == 0) {
            int s = 0;
            for (int q = 0; q < w; q++) s += ldi(gc + q);
            sbase = s;
          }
          __syncthreads();
          skel_before = sbase;
        }
      }
      // exs: skeleton columns before each grid index (grid order = storage order)
      {
        // the group's columns in grid order: a = w DQ_CPW + g + CS_NG j, so
        // order within the workgroup is (j, g); a block scan over
        // (j, g) pairs in that order
        int run = skel_before;
#pragma unroll
        for (int j = 0; j < DQ_CPG; j++) {
          const int a = w * DQ_CPW + g + CS_NG * j;
          const int is = (a < m && lb[j] < k && h == 0) ? 1 : 0;
          int64_t tot;
          const int ex = (int)block_excl_scan_i64<CS_NW>(is, &tot, sred);
          // (lane h = 0 of group g holds the column's flag: the scan over
          // threads in order is the scan over the groups in order)
          if (a < m && h == 0) sti(D.exs + A.selo[i] + a, run + ex);
          run += (int)tot;
        }
      }
      if (!meet()) {
        abort = true;
        break;
      }
      if (k == 0 || nr_ == 0) break;
      // R11 by columns into gR (each skeleton column's rows above its
      // position), R_tt and the pivot order are known to every workgroup
      for (int t = tid; t < k; t += CS_NT) rdg[t] = 1.0 / rdiag[t];
#pragma unroll
      for (int j = 0; j < DQ_CPG; j++) {
        const int la = lb[j];
        if (la < 0 || la >= k) continue;
#pragma unroll
        for (int u = 0; u < RL; u++) {
          const int r = CS_LPC * u + h;
          if (r < la) st(gR + (int64_t)la * k + r, col[j][u]);
        }
      }
      if (!meet()) {
        abort = true;
        break;
      }
      // back substitution in every column at once: a column at position
      // j < k solves R11 x = e_j (a column of R11^-1), one at a position
      // >= k solves R11 n = R12 e (a column of N, over its rows < k); R11
      // passes through LDS, RC columns at a time, last columns first
#pragma unroll
      for (int j = 0; j < DQ_CPG; j++) {
        const int la = lb[j];
        if (la >= 0 && la < k) {
#pragma unroll
          for (int u = 0; u < RL; u++) col[j][u] = (CS_LPC * u + h) == la ? 1.0 : 0.0;
        }
      }
      for (int j1 = k; j1 > 0; j1 -= RC) {
        const int j0 = j1 - RC > 0 ? j1 - RC : 0;
        __syncthreads();
        for (int e2 = tid; e2 < (j1 - j0) * CMAX; e2 += CS_NT) {
          const int jc = e2 / CMAX, r = e2 - jc * CMAX;
          Lr[e2] = r < j0 + jc ? ld(gR + (int64_t)(j0 + jc) * k + r) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ub = RL - 1; ub >= 0; ub--) {
          const int jlo = CS_LPC * ub > j0 ? CS_LPC * ub : j0;
          const int jhi = CS_LPC * ub + CS_LPC < j1 ? CS_LPC * ub + CS_LPC : j1;
          if (jlo >= jhi) continue;
#pragma unroll 1
          for (int jj = jhi - 1; jj >= jlo; jj--) {
            const int hj = jj - CS_LPC * ub;
            const double rdj = rdg[jj];
            const double *Rc = Lr + (int64_t)(jj - j0) * CMAX;
            double xv[DQ_CPG];
#pragma unroll
            for (int j = 0; j < DQ_CPG; j++) {
              xv[j] = __shfl(col[j][ub], (lane & ~(CS_LPC - 1)) + hj, WAVE) * rdj;
              if (h == hj) col[j][ub] = xv[j];
            }
#pragma unroll
            for (int u = 0; u <= ub; u++) {
              const int r = CS_LPC * u + h;
              if (r < jj) {
                const double rr = Rc[r];
#pragma unroll
                for (int j = 0; j < DQ_CPG; j++) col[j][u] = fma(-rr, xv[j], col[j][u]);
              }
            }
          }
        }
      }
      // R11^-1 by columns into gI; rinv_i = |row i of R11^-1| (a group per
      // row, lane h summing the columns jc = h (mod 16), then the group sum)
#pragma unroll
      for (int j = 0; j < DQ_CPG; j++) {
        const int la = lb[j];
        if (la < 0 || la >= k) continue;
#pragma unroll
        for (int u = 0; u < RL; u++) {
          const int r = CS_LPC * u + h;
          if (r < k) st(gI + (int64_t)la * k + r, col[j][u]);
        }
      }
      if (!meet()) {
        abort = true;
        break;
      }
      for (int ii = g; ii < k; ii += CS_NG) {
        double sq = 0.0;
        for (int jc = h; jc < k; jc += CS_LPC) {
          const double y = ld(gI + (int64_t)jc * k + ii);
          sq = fma(y, y, sq);
        }
        sq = g16_sum(sq);
        if (h == 0) rinv[ii] = sqrt(sq);
      }
      __syncthreads();
      // rho^2 arg-max over (i, j): ties smallest j, then i (pair j k + i);
      // G rows are written on every pass, the last leaves the final ones
      ArgMax am{-1.0, -1};
#pragma unroll
      for (int j = 0; j < DQ_CPG; j++) {
        const int a = w * DQ_CPW + g + CS_NG * j;
        const int la = lb[j];
        if (la < k) continue;  // (also the columns beyond m: la = -1)
        const double gam = sqrt(nr[j]);
        double *Gr = A.G_out + A.go[i] + (int64_t)(a - ldi(D.exs + A.selo[i] + a)) * k;
        const int base = (la - k) * k;
#pragma unroll
        for (int u = 0; u < RL; u++) {
          const int ii = CS_LPC * u + h;
          if (ii < k) {
            const double nv = col[j][u];
            const double gw = gam * rinv[ii];
            const double r2 = nv * nv + gw * gw;
            am = amax_pick(am, ArgMax{r2, base + ii});
            Gr[ldi(D.exs + A.selo[i] + piv[ii])] = nv;
          }
        }
      }
      am = block_argmax<CS_NW>(am, ared);
      int ws_ = 0, wa_ = -1;
      am = group_argmax(am, -1, 2, &ws_, &wa_);
      if (abort) break;
      if (!(sqrt(am.v) > A.f)) break;
      if (++nsw > 64 * k) {
        failed = true;
        break;
      }
      const int bj = am.a / k, bi = am.a % k;
#pragma unroll
      for (int j = 0; j < DQ_CPG; j++) {
        const int la = lb[j];
        if (la == bi)
          lb[j] = k + bj;
        else if (la == k + bj)
          lb[j] = bi;
      }
      __syncthreads();
      build(true);
      qr(false, k);
      if (abort) break;
    }
    if (abort) break;
    if (w == 0 && tid == 0 && nsw > 0) atomicAdd(A.swaps, nsw);
    // canonical output: skeleton indices ascending, then the rest
    int *sel = A.sel_out + A.selo[i];
#pragma unroll
    for (int j = 0; j < DQ_CPG; j++) {
      const int a = w * DQ_CPW + g + CS_NG * j;
      if (a >= m || h != 0) continue;
      if (failed) {
        sel[a] = a;
      } else {
        const int ex = ldi(D.exs + A.selo[i] + a);
        if (lb[j] < k)
          sel[ex] = a;
        else
          sel[k + (a - ex)] = a;
      }
    }
    if (failed && w == 0 && tid == 0) atomicOr(A.err, 1);
    if (w == 0 && tid == 0) A.k_out[i] = failed ? 0 : k;
  }
}

// Positions of the level's wide-form nodes (sorted by decreasing grid) per
// class: out[2q], out[2q+1] = [lo, hi) for class q = 0 (grids above
// DQ_MAXW * DQ_CPW, left to the streaming form) and q = 1 + s for nw =
// DQ_MAXW >> s (grids in (DQ_CPW * nw / 2, DQ_CPW * nw]; nw = 1: up to DQ_CPW).
__global__ void k_dq_ranges(const int *order, const int *cnt, const int *m, int *out) {
  constexpr int NC = 6;
  const int n = *cnt;
  if (threadIdx.x != 0) return;
  int e = 0;
  for (int q = 0; q < NC; q++) {
    // upper bound of class q's grids (class 0: none)
    const int lim = q == 0 ? DQ_MAXW * DQ_CPW : (DQ_MAXW >> (q - 1)) * DQ_CPW / 2;
    const int lo = e;
    if (q == NC - 1) {
      e = n;
    } else {
      while (e < n && m[order[e]] > lim) e++;
    }
    out[2 * q] = lo;
    out[2 * q + 1] = e;
  }
}

// Node order of a level for the wide form: grids larger than `lim` first,
// by decreasing size (a 16-bit key), then the rest; `big` counts the former.
__global__ void k_order_keys(int nb, int ne, const int *m, int lim, uint64_t *keys, int *vals,
                             int *big) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne - nb) return;
  const int mm = m[nb + e];
  const uint64_t sz = (uint64_t)(65535 - (mm < 65535 ? mm : 65535));
  keys[e] = (mm > lim ? 0ull : (1ull << 16)) | sz;
  vals[e] = nb + e;
  if (mm > lim) atomicAdd(big, 1);
}

// ------------------------------------------------------------------------
// HSS near-field SVD, one workgroup per node.  The kept left singular
// vectors of the block row A_i (m x nc; rows = this side's grid points) are
// the right singular vectors of B = A_i^T (nc x m), held row-major: B[t][c]
// is the kernel between grid point c and near-field point t.
//  (1) Householder QR of B with column pivoting: at step j the column with
//      the largest remaining norm is reduced; column norms are recomputed
//      exactly as the update writes them; columns stay in place, so the
//      first kq = min(m, nc) rows end up holding R P^T.
//  (2) One-sided (Hestenes) Jacobi on the rows of R P^T: parallel
//      round-robin pairs, a rotation wherever |a_p . a_q| > 1e-15 |a_p||a_q|,
//      sweeps until none rotates.  R P^T has B's right singular vectors, so
//      the converged rows, normalised, are the wanted vectors in the grid's
//      own point order and their norms are the singular values; no rotation
//      matrix is accumulated.  The pivoted factor has graded rows, on which
//      the sweeps settle in about a third of the count they need on A_i.
//  (3) Vectors with sigma >= eps * sigma_1, by decreasing sigma (ties: row),
//      are written as S (m x ks row-major).
// Threads: the QR maps lanes to columns (coalesced rows of B) and, for
// m <= 128, splits the rows t over G = 256 / CP segments whose partial dots
// and norms meet in LDS; the Jacobi gives each pair SV_G lanes.
// ------------------------------------------------------------------------
constexpr int SV_NT = 256, SV_G = 8, SV_MMAX = 1024;  // largest grid of a node

struct SvdArgs {
  int nb, ne;
  const int *m_me;
  const int64_t *gbeg_me;
  const int *slot_me;
  const double *P_me;
  const int *m_ot;
  const int64_t *gbeg_ot;
  const int *slot_ot;
  const double *P_ot;
  const int *Nrow, *Ncol;
  int rowside;
  int kid, d;
  double diag, eps;
  double *scratch;  // per workgroup: B ((ncmax + 1) x ldb) when it is not in LDS
  int64_t wg_stride;
  double *S;  // output
  const int64_t *S_off;
  int *ks_out;
  int *ks_max;       // largest ks of the launch
  const double *pd;  // double-layer kernel: per-point data by point id (X = Y)
};

// Small per-node arrays at the front of the dynamic LDS (in doubles):
// norm partials (two buffers of NP), dot partials (SV_NT), beta (mp), then
// pivot step and pivot column (mp ints each).  B follows when it is in LDS.
__host__ __device__ inline int svd_np(int mp) { return mp > SV_NT ? mp : SV_NT; }
__host__ __device__ inline int svd_small(int mp) { return 2 * svd_np(mp) + SV_NT + 2 * mp; }

template <int NCL, bool LDS>
__global__ void __launch_bounds__(SV_NT) k_near_svd(SvdArgs A, int mpx, int ldl) {
  extern __shared__ double dyn_svd[];
  __shared__ int any_rot;
  const int tid = threadIdx.x, lane = tid & 63;
  const int NP = svd_np(mpx);
  double *pnrm = dyn_svd;                 // [2][NP]
  double *pdot = dyn_svd + 2 * NP;        // [SV_NT]
  double *beta = pdot + SV_NT;            // [mp]
  int *piv = (int *)(beta + mpx);         // [mp]
  int *pcol = piv + mpx;                  // [mp]
  double *sg = pnrm;                      // after the QR: singular values
  int *ord = (int *)beta;                 // after the QR: order by sigma
  double *Bm = LDS ? dyn_svd + svd_small(mpx) : A.scratch + (int64_t)blockIdx.x * A.wg_stride;
  for (int i = A.nb + blockIdx.x; i < A.ne; i += gridDim.x) {
    const int m = A.m_me[i];
    int nc = 0;
    for (int q = A.Nrow[i]; q < A.Nrow[i + 1]; q++) nc += A.m_ot[A.Ncol[q]];
    const int ldb = LDS ? ldl : m;
    __syncthreads();
    if (m == 0 || nc == 0) {
      if (tid == 0) A.ks_out[i] = 0;
      continue;
    }
    // columns per pass and row segments: G * CP = SV_NT
    const int CP = m <= 64 ? 64 : m <= 128 ? 128 : SV_NT;
    const int G = SV_NT / CP;
    const int g = tid / CP, cl = tid % CP;
    // B = A_i^T: row t <-> point of the other side's grid, N_i order
    {
      int o = 0;
      for (int q = A.Nrow[i]; q < A.Nrow[i + 1]; q++) {
        const int j = A.Ncol[q];
        const int mj = A.m_ot[j];
        const int64_t gj = A.gbeg_ot[j];
        for (int e = tid; e < mj * m; e += SV_NT) {
          const int b = e / m, c = e % m;
          const int64_t ime = A.slot_me[A.gbeg_me[i] + c], iot = A.slot_ot[gj + b];
          const double *pme = A.P_me + ime * A.d;
          const double *pot = A.P_ot + iot * A.d;
          const double *dme = A.pd ? A.pd + 3 * ime : nullptr;
          const double *dot = A.pd ? A.pd + 3 * iot : nullptr;
          Bm[(int64_t)(o + b) * ldb + c] = A.rowside
                                               ? kernel_f64(A.kid, pme, pot, A.d, A.diag, dme, dot)
                                               : kernel_f64(A.kid, pot, pme, A.d, A.diag, dot, dme);
        }
        o += mj;
      }
    }
    for (int c = tid; c < m; c += SV_NT) piv[c] = -1;
    __syncthreads();
    // column norm partials over rows t = g (mod G)
    for (int c = cl; c < m; c += CP) {
      double s = 0.0;
      for (int t = g; t < nc; t += G) {
        const double v = Bm[(int64_t)t * ldb + c];
        s = fma(v, v, s);
      }
      pnrm[g * m + c] = s;
    }
    __syncthreads();
    // (1) pivoted Householder QR of B
    const int kmax = m < nc ? m : nc;
    int kq = kmax;
    for (int j = 0; j < kmax; j++) {
      const double *pn = pnrm + (j & 1) * NP;
      double *pw = pnrm + ((j + 1) & 1) * NP;
      // arg-max of the remaining column norms, the same in every wave
      double best = -1.0;
      int bi = 0x7fffffff;
      for (int c = lane; c < m; c += 64) {
        const int pv = piv[c];
        if (pv >= 0 && pv < j) continue;
        double v = 0.0;
        for (int h = 0; h < G; h++) v += pn[h * m + c];
        if (v > best) {
          best = v;
          bi = c;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (!(best > 0.0)) {  // every remaining column is zero
        kq = j;
        break;
      }
      const int p = bi;
      const double al = Bm[(int64_t)j * ldb + p];
      const double sig = sqrt(best);
      const double be = al >= 0.0 ? -sig : sig;
      const double u0 = al - be;
      const double cf = 1.0 / (sig * (sig + fabs(al)));
      if (tid == 0) {
        beta[j] = be;
        pcol[j] = p;
      }
      const int gj = j % G;
      const int t0 = j + 1 + ((g - (j + 1) % G) + G) % G;  // first t > j with t = g (mod G)
      double wr[SV_MMAX / SV_NT];  // this thread's dots when G == 1
#pragma unroll
      for (int u = 0; u < SV_MMAX / SV_NT; u++) {
        const int c = cl + u * CP;
        if (c >= m) break;
        double w = 0.0;
        if (c != p && piv[c] < 0) {
          if (g == gj) w = u0 * Bm[(int64_t)j * ldb + c];
          for (int t = t0; t < nc; t += G)
            w = fma(Bm[(int64_t)t * ldb + p], Bm[(int64_t)t * ldb + c], w);
        }
        if (G > 1)
          pdot[g * m + c] = w;
        else
          wr[u] = w;
      }
      if (G > 1) __syncthreads();
#pragma unroll
      for (int u = 0; u < SV_MMAX / SV_NT; u++) {
        const int c = cl + u * CP;
        if (c >= m) break;
        if (c == p) {
          if (g == 0) piv[p] = j;
          continue;
        }
        if (piv[c] >= 0) continue;
        double w;
        if (G > 1) {
          w = 0.0;
          for (int h = 0; h < G; h++) w += pdot[h * m + c];
        } else {
          w = wr[u];
        }
        const double f = cf * w;
        if (g == gj) Bm[(int64_t)j * ldb + c] = fma(-f, u0, Bm[(int64_t)j * ldb + c]);
        double nr = 0.0;
        for (int t = t0; t < nc; t += G) {
          const double v = fma(-f, Bm[(int64_t)t * ldb + p], Bm[(int64_t)t * ldb + c]);
          Bm[(int64_t)t * ldb + c] = v;
          nr = fma(v, v, nr);
        }
        pw[g * m + c] = nr;
      }
      __syncthreads();
    }
    // R P^T in rows [0, kq): each pivot column holds beta at its step and
    // zeros below it; an odd kq gets a zero pad row for the pairing
    const int kp = kq + (kq & 1);
    for (int e = tid; e < kq * kp; e += SV_NT) {
      const int j = e / kp, t = e % kp;
      const int pc = pcol[j];
      if (t == j)
        Bm[(int64_t)t * ldb + pc] = beta[j];
      else if (t > j)
        Bm[(int64_t)t * ldb + pc] = 0.0;
    }
    if (kq & 1)
      for (int c = tid; c < m; c += SV_NT) {
        int pv = piv[c];
        if (pv < 0) Bm[(int64_t)kq * ldb + c] = 0.0;  // pivot columns are zeroed above
      }
    __syncthreads();
    // (2) Jacobi sweeps on the rows of R P^T
    const int gi = tid / SV_G, gl = tid % SV_G;
    const int npairs = kp / 2;
    for (int sweep = 0; sweep < 80 && kq > 1; sweep++) {
      if (tid == 0) any_rot = 0;
      __syncthreads();
      for (int round = 0; round < kp - 1; round++) {
        for (int pr = gi; pr < npairs; pr += SV_NT / SV_G) {
          // round-robin: position 0 fixed, the others rotate
          const int a0 = pr, b0 = kp - 1 - pr;
          auto rr = [&](int x) { return x == 0 ? 0 : 1 + (x - 1 + round) % (kp - 1); };
          int pp = rr(a0), qq = rr(b0);
          if (pp > qq) {
            const int t = pp;
            pp = qq;
            qq = t;
          }
          double *ap = Bm + (int64_t)pp * ldb, *aq = Bm + (int64_t)qq * ldb;
          double al = 0.0, be = 0.0, ga = 0.0;
          double xr[NCL > 0 ? NCL : 1], yr[NCL > 0 ? NCL : 1];
          if constexpr (NCL > 0) {
#pragma unroll
            for (int v = 0; v < NCL; v++) {
              const int t = gl + SV_G * v;
              const int tc = t < m ? t : 0;
              xr[v] = ap[tc];
              yr[v] = aq[tc];
            }
#pragma unroll
            for (int v = 0; v < NCL; v++) {
              if (gl + SV_G * v < m) {
                al = fma(xr[v], xr[v], al);
                be = fma(yr[v], yr[v], be);
                ga = fma(xr[v], yr[v], ga);
              }
            }
          } else {
            for (int t = gl; t < m; t += SV_G) {
              const double x = ap[t], y = aq[t];
              al = fma(x, x, al);
              be = fma(y, y, be);
              ga = fma(x, y, ga);
            }
          }
          static_assert(SV_G == 8, "pair sums are 8-lane DPP sums");
          al = g8_sum(al);
          be = g8_sum(be);
          ga = g8_sum(ga);
          if (al == 0.0 || be == 0.0) continue;
          if (fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
          if (gl == 0) any_rot = 1;
          const double zeta = (be - al) / (2.0 * ga);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + tt * tt);
          const double sn = cs * tt;
          if constexpr (NCL > 0) {
#pragma unroll
            for (int v = 0; v < NCL; v++) {
              const int t = gl + SV_G * v;
              if (t < m) {
                ap[t] = cs * xr[v] - sn * yr[v];
                aq[t] = sn * xr[v] + cs * yr[v];
              }
            }
          } else {
            for (int t = gl; t < m; t += SV_G) {
              const double x = ap[t], y = aq[t];
              ap[t] = cs * x - sn * y;
              aq[t] = sn * x + cs * y;
            }
          }
        }
        __syncthreads();
      }
      if (!any_rot) break;
      __syncthreads();
    }
    // (3) singular values = row norms; order by decreasing sigma (ties: row)
    for (int a = tid; a < kq; a += SV_NT) {
      double s = 0.0;
      for (int t = 0; t < m; t++) s = fma(Bm[(int64_t)a * ldb + t], Bm[(int64_t)a * ldb + t], s);
      sg[a] = sqrt(s);
    }
    __syncthreads();
    for (int a = tid; a < kq; a += SV_NT) {
      int rank = 0;
      for (int b = 0; b < kq; b++)
        if (sg[b] > sg[a] || (sg[b] == sg[a] && b < a)) rank++;
      ord[rank] = a;
    }
    __syncthreads();
    const double s1 = kq > 0 ? sg[ord[0]] : 0.0;
    int ks = 0;
    if (s1 > 0.0)
      for (int a = 0; a < kq; a++)
        if (sg[ord[a]] >= A.eps * s1) ks = a + 1;
    double *S = A.S + A.S_off[i - A.nb];
    for (int e = tid; e < m * ks; e += SV_NT) {
      const int r = e / ks, q = e % ks;
      const int a = ord[q];
      S[e] = Bm[(int64_t)a * ldb + r] / sg[a];
    }
    if (tid == 0) {
      A.ks_out[i] = ks;
      atomicMax(A.ks_max, ks);
    }
  }
}

// ------------------------------------------------------------------------
// level bookkeeping
// ------------------------------------------------------------------------
struct PrepArgs {
  int nb, ne;
  const int *nchild, *first_child;
  const int *xb, *xe;  // point range of this side
  int *m;
  int64_t *gbeg;
  const int *k;
  const int64_t *hbeg;
  int c0, hss;
  int64_t *cm, *cg;  // out: m and G capacity per node (for scans)
  int *mmax;
};

__global__ void k_leaf_init(int nnodes, const int *nchild, const int *xb, const int *xe, int *m,
                            int64_t *gbeg, int *k) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnodes) return;
  if (i == 0) {
    m[0] = 0;
    k[0] = 0;
    gbeg[0] = 0;
  } else if (nchild[i] == 0) {
    m[i] = xe[i] - xb[i];
    gbeg[i] = xb[i];
  }
}

// Leaf count (nodes without children) into *cnt (zeroed before).
__global__ void k_count_leaves(int nnodes, const int *nchild, int *cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool leaf = i < nnodes && nchild[i] == 0;
  const uint64_t b = __ballot(leaf);
  if ((threadIdx.x & (WAVE - 1)) == 0 && b) atomicAdd(cnt, (int)__popcll(b));
}

__global__ void k_level_prep(PrepArgs A) {
  int i = A.nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.ne) return;
  int m;
  if (A.nchild[i] > 0) {
    int fc = A.first_child[i];
    m = 0;
    for (int c = 0; c < A.nchild[i]; c++) m += A.k[fc + c];
    A.m[i] = m;
    A.gbeg[i] = A.hbeg[fc];
  } else {
    m = A.m[i];
  }
  int64_t mm = m;
  int64_t cap;
  if (A.hss)
    cap = mm * mm / 4;
  else
    cap = (2 * A.c0 >= mm) ? mm * mm / 4 : (mm - A.c0) * A.c0;
  A.cm[i - A.nb] = mm;
  A.cg[i - A.nb] = cap;
  atomicMax(A.mmax, m);
}

// One workgroup for a whole level of at most LV_NT * LV_PER nodes: the grid
// sizes and G capacities (as k_level_prep), their exclusive scans into selo
// and go (relative to the level), and the totals for the host read -- one
// launch instead of a prep kernel, two scans and two offset writes.
constexpr int LV_NT = 1024, LV_PER = 4;
__device__ __forceinline__ int64_t level_cap(int64_t mm, int c0, int hss) {
  if (hss) return mm * mm / 4;
  return (2 * c0 >= mm) ? mm * mm / 4 : (mm - c0) * c0;
}
__global__ void __launch_bounds__(LV_NT) k_level_prep1(PrepArgs A, int64_t *selo, int64_t *go,
                                                       int64_t *tot) {
  __shared__ int64_t lds[LV_NT / WAVE + 1];
  __shared__ int smax;
  if (threadIdx.x == 0) smax = 0;
  const int i0 = A.nb + threadIdx.x * LV_PER;
  int64_t mv[LV_PER], cv[LV_PER], sm = 0, sg = 0;
  int mx = 0;
#pragma unroll
  for (int u = 0; u < LV_PER; u++) {
    const int i = i0 + u;
    mv[u] = cv[u] = 0;
    if (i < A.ne) {
      int m;
      if (A.nchild[i] > 0) {
        const int fc = A.first_child[i];
        m = 0;
        for (int c = 0; c < A.nchild[i]; c++) m += A.k[fc + c];
        A.m[i] = m;
        A.gbeg[i] = A.hbeg[fc];
      } else {
        m = A.m[i];
      }
      mx = max(mx, m);
      mv[u] = m;
      cv[u] = level_cap(m, A.c0, A.hss);
    }
    sm += mv[u];
    sg += cv[u];
  }
  int64_t tm, tg;
  int64_t om = block_excl_scan_i64<LV_NT / WAVE>(sm, &tm, lds);
  int64_t og = block_excl_scan_i64<LV_NT / WAVE>(sg, &tg, lds);
#pragma unroll
  for (int u = 0; u < LV_PER; u++) {
    const int i = i0 + u;
    if (i < A.ne) {
      selo[i] = om;
      go[i] = og;
    }
    om += mv[u];
    og += cv[u];
  }
  if (mx > 0) atomicMax(&smax, mx);  // smax was set before the scans' barriers
  __syncthreads();
  if (threadIdx.x == 0) {
    tot[0] = tm;
    tot[1] = tg;
    *A.mmax = smax;  // the level's largest grid (no zeroing needed before)
  }
}

// One workgroup for a whole level (as above): the skeleton slots of the
// level's nodes, hbeg = running slot count + exclusive scan of k, and the
// running count advanced by the level's total (kept on the device).
__global__ void __launch_bounds__(LV_NT) k_level_slots1(int nb, int ne, const int *k,
                                                        int64_t *hbeg, int64_t *run) {
  __shared__ int64_t lds[LV_NT / WAVE + 1];
  const int i0 = nb + threadIdx.x * LV_PER;
  int64_t kv[LV_PER], sk = 0;
#pragma unroll
  for (int u = 0; u < LV_PER; u++) {
    const int i = i0 + u;
    kv[u] = i < ne ? k[i] : 0;
    sk += kv[u];
  }
  int64_t tk;
  const int64_t base = *run;
  int64_t o = base + block_excl_scan_i64<LV_NT / WAVE>(sk, &tk, lds);
#pragma unroll
  for (int u = 0; u < LV_PER; u++) {
    const int i = i0 + u;
    if (i < ne) hbeg[i] = o;
    o += kv[u];
  }
  if (threadIdx.x == 0) *run = base + tk;
}

__global__ void k_kcopy(int nb, int ne, const int *k, int64_t *out) {
  int i = nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ne) out[i - nb] = k[i];
}

__global__ void k_set_hbeg(int nb, int ne, const int64_t *off, int64_t *hbeg) {
  int i = nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ne) hbeg[i] = off[i - nb];
}

__global__ void k_set_rel(int nb, int ne, const int64_t *off, int64_t *dst) {
  int i = nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ne) dst[i] = off[i - nb];
}

// skeleton slots: slot_id[hbeg + t] = slot_id[gbeg + sel[t]]
__global__ void k_slot_ids(int nb, int ne, const int *k, const int64_t *hbeg,
                           const int64_t *gbeg, const int64_t *selo, const int *sel,
                           int *slot_id) {
  int i = nb + blockIdx.x;
  if (i >= ne) return;
  const int *s = sel + selo[i];
  for (int t = threadIdx.x; t < k[i]; t += blockDim.x)
    slot_id[hbeg[i] + t] = slot_id[gbeg[i] + s[t]];
}

__global__ void k_iota(int *a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int)i;
}

__global__ void k_near_cols(int nb, int ne, const int *Nrow, const int *Ncol, const int *m_ot,
                            const int *m_me, int *ncmax, int64_t *s_cap) {
  int i = nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  int nc = 0;
  for (int q = Nrow[i]; q < Nrow[i + 1]; q++) nc += m_ot[Ncol[q]];
  atomicMax(ncmax, nc);
  int64_t mm = m_me[i];
  s_cap[i - nb] = mm * mm;
}

// G (m-k) x k  ->  G^T k x (m-k), one workgroup per node
__global__ void k_transpose_G(int nb, int ne, const int *m, const int *k, const int64_t *go,
                              const double *G, double *Gt) {
  int i = nb + blockIdx.x;
  if (i >= ne) return;
  const int kk = k[i], nr = m[i] - kk;
  const double *src = G + go[i];
  double *dst = Gt + go[i];
  for (int e = threadIdx.x; e < nr * kk; e += blockDim.x) {
    int a = e / kk, t = e - a * kk;
    dst[(int64_t)t * nr + a] = src[e];
  }
}

// BF16 copies of G for the matrix-core product (layouts in LevelSide)
__global__ void k_gb_sizes(int nb, int ne, const int *m, const int *k, int64_t *cu, int64_t *cd) {
  int i = nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  const int kk = k[i], nr = m[i] - kk;
  cu[i - nb] = (int64_t)kk * ((nr + 7) & ~7);
  cd[i - nb] = (int64_t)nr * ((kk + 7) & ~7);
}

__global__ void __launch_bounds__(256) k_g_to_bf16(int nb, int ne, const int *m, const int *k,
                                                   const int64_t *go, const double *G,
                                                   const int64_t *gobu, const int64_t *gobd,
                                                   unsigned short *Gbu, unsigned short *Gbd) {
  const int i = nb + blockIdx.x;
  if (i >= ne) return;
  const int kk = k[i], nr = m[i] - kk;
  if (kk == 0 || nr == 0) return;
  const double *Gi = G + go[i];  // (m-k) x k row-major
  const int nr8 = (nr + 7) & ~7, k8 = (kk + 7) & ~7;
  unsigned short *U = Gbu + gobu[i], *D = Gbd + gobd[i];
  for (int q = threadIdx.x; q < kk * nr8; q += blockDim.x) {
    const int a8 = q / (kk * 8), r = q - a8 * kk * 8, t = r >> 3, a = a8 * 8 + (r & 7);
    U[q] = bf16_bits(a < nr ? (float)Gi[(int64_t)a * kk + t] : 0.0f);
  }
  for (int q = threadIdx.x; q < nr * k8; q += blockDim.x) {
    const int t8 = q / (nr * 8), r = q - t8 * nr * 8, a = r >> 3, t = t8 * 8 + (r & 7);
    D[q] = bf16_bits(t < kk ? (float)Gi[(int64_t)a * kk + t] : 0.0f);
  }
}

__global__ void k_to_f32(const double *in, float *out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

// ------------------------------------------------------------------------
__global__ void k_zero_side(int nn, int *m, int *k, int *ks, int64_t *hbeg, int64_t *selo,
                            int64_t *go) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  m[i] = k[i] = ks[i] = 0;
  hbeg[i] = selo[i] = go[i] = 0;
}

static void alloc_side(Handle &h, Side &S) {
  int nn = h.nnodes;
  S.m = h.mem.alloc_n<int>(nn);
  S.k = h.mem.alloc_n<int>(nn);
  S.ks = h.mem.alloc_n<int>(nn);
  S.gbeg = h.mem.alloc_n<int64_t>(nn);
  S.hbeg = h.mem.alloc_n<int64_t>(nn);
  S.selo = h.mem.alloc_n<int64_t>(nn);
  S.go = h.mem.alloc_n<int64_t>(nn);
  k_zero_side<<<ceil_div(nn, 256), 256, 0, h.stream>>>(nn, S.m, S.k, S.ks, S.hbeg, S.selo, S.go);
  SMASH_CHECK_LAUNCH();
  S.lv.assign(h.nlevels + 1, LevelSide{});
}

static void grow_slots(Handle &h, Side &S, int64_t need) {
  if (need <= S.slot_cap) return;
  int64_t nc = S.slot_cap > 0 ? S.slot_cap : 1024;
  while (nc < need) nc *= 2;
  int *q = h.mem.alloc_n<int>(nc);
  if (S.slot_id)
    SMASH_HIP(hipMemcpyAsync(q, S.slot_id, sizeof(int) * S.nslots, hipMemcpyDeviceToDevice, h.stream));
  S.slot_id = q;
  S.slot_cap = nc;
}

struct SideCtx {
  Side *S;
  bool rowside;
  const int *xb, *xe;
  const double *P;
  int64_t n;
  // per level
  int64_t *cm = nullptr, *cg = nullptr;
  int mmax = 0;
  double *Svec = nullptr;
  int64_t *S_off = nullptr;
  bool gt_first = false;  // compr wrote G^T (the register kernel)
  int c0 = 0;             // basis width p^d, or 2 p^d (double-layer column side)
  int *ks_max = nullptr;  // HSS: device word, the level's largest SVD rank
};

void build_generators(Handle &h) {
  hipStream_t s = h.stream;
  DeviceArena tmp, keep;  // per-level temporaries; counters for the whole build
  tmp.stream = s;
  keep.stream = s;
  try {
    const int pd = [&] {
      int c = 1;
      for (int t = 0; t < h.d; t++) c *= h.p;
      return c;
    }();
    const bool dl = h.kid == SMASH_KERNEL_DOUBLE_LAYER;
    if (h.p > ID_PMAX) throw Error{SMASH_E_INVALID_ARG, "interpolation order above 64"};
    if ((dl ? 2 * pd : pd) > ID_CMAX)
      throw Error{SMASH_E_UNSUPPORTED, "basis width above 512"};
    const bool hss = h.adm == SMASH_ADM_WEAK;
    alloc_side(h, h.row);
    h.col = h.reuse ? &h.row : &h.col_own;
    if (!h.reuse) alloc_side(h, h.col_own);
    std::vector<SideCtx> sides;
    sides.push_back(SideCtx{&h.row, true, h.xb, h.xe, h.Xp, h.nx});
    if (!h.reuse) sides.push_back(SideCtx{&h.col_own, false, h.yb, h.ye, h.Yp, h.ny});
    // the double layer's column basis: each Lagrange column times m_1 and m_2
    for (auto &sc : sides) sc.c0 = (dl && !sc.rowside) ? 2 * pd : pd;
    int nn = h.nnodes;
    // slot capacity for every level at once: a level's grids are disjoint
    // sets of points, so it adds at most min(n, nodes * c) skeleton slots
    // (HSS: at most n); the running slot count stays on the device
    for (auto &sc : sides) {
      Side &S = *sc.S;
      int64_t bound = sc.n + 1024;
      for (int l = 2; l <= h.nlevels; l++) {
        const int64_t nl = h.level_beg[l] - h.level_beg[l - 1];
        bound += hss ? sc.n : std::min<int64_t>(sc.n, nl * sc.c0);
      }
      grow_slots(h, S, bound);
      k_iota<<<ceil_div(sc.n, 256), 256, 0, s>>>(S.slot_id, sc.n);
      SMASH_CHECK_LAUNCH();
      S.nslots = sc.n;
      k_leaf_init<<<ceil_div(nn, 256), 256, 0, s>>>(nn, h.nchild, sc.xb, sc.xe, S.m, S.gbeg, S.k);
      SMASH_CHECK_LAUNCH();
    }
    int *dmax = keep.alloc_n<int>(4);  // largest grid, near width, SVD rank per side
    int *dsw = keep.alloc_n<int>(3);  // swaps, cap flag, leaves
    int64_t *dslots = keep.alloc_n<int64_t>(2);  // running slot count per side
    for (size_t q = 0; q < sides.size(); q++) set_i64(dslots + q, sides[q].S->nslots, s);
    SMASH_HIP(hipMemsetAsync(dsw, 0, 3 * sizeof(int), s));
    k_count_leaves<<<ceil_div(nn, 256), 256, 0, s>>>(nn, h.nchild, dsw + 2);
    SMASH_CHECK_LAUNCH();
    int dev_cus = 256, dev_lds = 64 * 1024;
    if (hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, h.device) !=
        hipSuccess)
      dev_cus = 256;
    if (hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h.device) !=
        hipSuccess)
      dev_lds = 64 * 1024;
    for (int l = h.nlevels; l >= 2; l--) {
      const int nb = h.level_beg[l - 1], ne = h.level_beg[l], nl = ne - nb;
      // (a) grids and capacities of both sides
      for (auto &sc : sides) {
        Side &S = *sc.S;
        sc.cm = tmp.alloc_n<int64_t>(nl);
        sc.cg = tmp.alloc_n<int64_t>(nl);
        PrepArgs pa{nb, ne, h.nchild, h.first_child, sc.xb, sc.xe, S.m, S.gbeg, S.k, S.hbeg, sc.c0,
                    hss ? 1 : 0, sc.cm, sc.cg, dmax};
        const int64_t *tot_m, *tot_g;
        if (nl <= LV_NT * LV_PER) {
          // the whole level in one workgroup
          int64_t *tot = tmp.alloc_n<int64_t>(2);
          k_level_prep1<<<1, LV_NT, 0, s>>>(pa, S.selo, S.go, tot);
          SMASH_CHECK_LAUNCH();
          tot_m = tot;
          tot_g = tot + 1;
        } else {
          SMASH_HIP(hipMemsetAsync(dmax, 0, sizeof(int), s));
          k_level_prep<<<ceil_div(nl, 256), 256, 0, s>>>(pa);
          SMASH_CHECK_LAUNCH();
          int64_t *o1 = tmp.alloc_n<int64_t>(nl + 1), *o2 = tmp.alloc_n<int64_t>(nl + 1);
          scan_i64(sc.cm, o1, nl, nullptr, s, tmp);
          scan_i64(sc.cg, o2, nl, nullptr, s, tmp);
          k_set_rel<<<ceil_div(nl, 256), 256, 0, s>>>(nb, ne, o1, S.selo);
          SMASH_CHECK_LAUNCH();
          k_set_rel<<<ceil_div(nl, 256), 256, 0, s>>>(nb, ne, o2, S.go);
          SMASH_CHECK_LAUNCH();
          tot_m = o1 + nl;
          tot_g = o2 + nl;
        }
        const int64_t *pin = pick_words(s, {{tot_m, 8}, {tot_g, 8}, {dmax, 4}});
        const int64_t hv[2] = {pin[0], pin[1]};
        const int mx = (int)pin[2];
        sc.mmax = mx;
        LevelSide &L = S.lv[l];
        L.sel_n = hv[0];
        L.g_n = hv[1];
        L.sel = h.mem.alloc_n<int>(hv[0]);
        L.G = h.mem.alloc_n<double>(hv[1]);
        L.Gt = h.mem.alloc_n<double>(hv[1]);
      }
      // (b) HSS: near-field SVD of each side
      if (hss) {
        for (size_t q = 0; q < sides.size(); q++) {
          SideCtx &sc = sides[q];
          SideCtx &ot = sides.size() > 1 ? sides[1 - q] : sides[0];
          Side &S = *sc.S;
          Side &O = *ot.S;
          int64_t *scap = tmp.alloc_n<int64_t>(nl), *soff = tmp.alloc_n<int64_t>(nl + 1);
          sc.ks_max = dmax + 2 + (int)q;
          SMASH_HIP(hipMemsetAsync(dmax + 1, 0, sizeof(int), s));
          SMASH_HIP(hipMemsetAsync(sc.ks_max, 0, sizeof(int), s));
          k_near_cols<<<ceil_div(nl, 256), 256, 0, s>>>(nb, ne, h.Nrow, h.Ncol, O.m, S.m, dmax + 1,
                                                        scap);
          SMASH_CHECK_LAUNCH();
          scan_i64(scap, soff, nl, nullptr, s, tmp);
          const int64_t *pin = pick_words(s, {{soff + nl, 8}, {dmax + 1, 4}});
          const int64_t stot = pin[0];
          const int ncmax = (int)pin[1];
          if (sc.mmax > SV_MMAX)
            throw Error{SMASH_E_UNSUPPORTED, "HSS grid larger than " + std::to_string(SV_MMAX) +
                                                 " points (raise leaf resolution)"};
          sc.Svec = tmp.alloc_n<double>(stot);
          sc.S_off = soff;
          const int mp = sc.mmax + (sc.mmax & 1);
          const int ncm = ncmax > 0 ? ncmax : 1;
          // B ((ncmax + 1) rows, odd row stride) after the small arrays in
          // LDS when it fits, else in a global tile per workgroup
          const int ldl = (sc.mmax > 0 ? sc.mmax : 1) | 1;
          const size_t sh_small = sizeof(double) * (size_t)svd_small(mp);
          const size_t sh_all = sh_small + sizeof(double) * (size_t)(ncm + 1) * ldl;
          const bool lds = sh_all <= (size_t)dev_lds;
          const int64_t wg_stride = lds ? 0 : (int64_t)(ncm + 1) * (sc.mmax > 0 ? sc.mmax : 1) + 8;
          int nwg = nl < 4 * dev_cus ? nl : 4 * dev_cus;
          if (!lds) {  // at most 2 GiB of tiles
            const int64_t cap = ((int64_t)1 << 28) / wg_stride;
            if (nwg > cap) nwg = cap > 0 ? (int)cap : 1;
          }
          double *scr = lds ? nullptr : tmp.alloc_n<double>((size_t)wg_stride * nwg);
          SvdArgs sa{nb, ne, S.m, S.gbeg, S.slot_id, sc.P, O.m, O.gbeg, O.slot_id, ot.P, h.Nrow,
                     h.Ncol, sc.rowside ? 1 : 0, h.kid, h.d, h.diag, h.eps_svd, scr,
                     wg_stride, sc.Svec, soff, S.ks, sc.ks_max, h.Ap};
          PhaseTimer pt(h, SMASH_PHASE_NEAR_SVD, s);
          // register-staged rotations when a pair's rows fit
          const int ncl = mp <= 64 ? 8 : mp <= 128 ? 16 : mp <= 256 ? 32 : 0;
          auto svd = [&](int grid) {
#define SMASH_SVD_CASE(NC)                                                          \
  if (ncl == NC) {                                                                  \
    if (lds)                                                                        \
      k_near_svd<NC, true><<<grid, SV_NT, sh_all, s>>>(sa, mp, ldl);                \
    else                                                                            \
      k_near_svd<NC, false><<<grid, SV_NT, sh_small, s>>>(sa, mp, 0);               \
  }
            SMASH_SVD_CASE(0) SMASH_SVD_CASE(8) SMASH_SVD_CASE(16) SMASH_SVD_CASE(32)
#undef SMASH_SVD_CASE
            SMASH_CHECK_LAUNCH();
          };
          if (h.batched) {
            svd(lds ? std::min(nl, 4 * dev_cus) : nwg);
          } else {
            for (int i = nb; i < ne; i++) {
              sa.nb = i;
              sa.ne = i + 1;
              sa.S_off = soff + (i - nb);
              svd(1);
            }
          }
        }
      }
      // (c) compr on each side
      for (auto &sc : sides) {
        Side &S = *sc.S;
        LevelSide &L = S.lv[l];
        // basis width: c0 interpolation columns plus, for HSS, the near
        // vectors (at most the grid size; their actual count is read back
        // only when that bound is above the limit)
        int cmax = sc.c0 + (hss ? sc.mmax : 0);
        if (hss && cmax > ID_CMAX) cmax = sc.c0 + (int)pick_words(s, {{sc.ks_max, 4}})[0];
        if (cmax > ID_CMAX) throw Error{SMASH_E_UNSUPPORTED, "basis width above 512"};
        // The register form (k_compr_w: the grid in registers, two lanes per
        // grid point) takes grids of up to 256 points when c <= 64; larger
        // grids and wider bases take the wide form (k_compr_s), largest
        // grids first.  A level may use both.
        constexpr int lpc = 4, cpg = 2;  // lanes per column group, columns per group
        const int mreg = std::min(sc.mmax, 256);
        const int mw = std::max(mreg, 1) * lpc / cpg;
        const int nt = mw <= 64 ? 64 : mw <= 128 ? 128 : mw <= 256 ? 256 : 512;
        const int cm = cmax <= 32 ? 32 : cmax <= 64 ? 64 : 0;
        const size_t shw = sizeof(double) * std::max((size_t)h.d * h.p * (nt / lpc * cpg),
                                                     (size_t)cm * (cm + 1));
        // (dynamic LDS plus at most 8 KB of static LDS within the device limit)
        const bool reg_ok = cm > 0 && cm <= nt && h.d * h.p <= nt && shw <= 64 * 1024 &&
                            shw + 8 * 1024 <= (size_t)dev_lds;
        const bool all_reg = reg_ok && sc.mmax <= 256;
        // the wide form: basis rows up to cw, tile columns of ldc rows; the
        // LDS left after its fixed parts holds the tile of grids of up to
        // lds_cols points
        // (224: the 6^3-point basis of 3D p = 6 without a sixth of idle rows)
        const int cw = cmax <= 64 ? 64 : cmax <= 128 ? 128 : cmax <= 224 ? 224 : cmax <= 256 ? 256 : 512;
        const int ldc = (cmax + 15) / 16 * 16;
        const size_t st_lds = sizeof(double) * (5 * ID_PMAX + 3 * cw) +
                              sizeof(int) * (cw + 2 * CS_NW) + sizeof(ArgMax) * (3 * CS_NW + 1) +
                              sizeof(int64_t) * (CS_NW + 1) + 512;
        const size_t fixed = sizeof(double) * (2 * CS_NW * (size_t)ldc + CS_NG * h.d * h.p);
        const size_t per_col = sizeof(double) * ((size_t)ldc + 2);
        int lds_cols = 0;
        if ((size_t)dev_lds > st_lds + fixed)
          lds_cols = (int)std::min<size_t>(((size_t)dev_lds - st_lds - fixed) / per_col,
                                           (size_t)sc.mmax);
        const size_t shs = fixed + per_col * (size_t)lds_cols;
        IdArgs ia{nb, ne, h.lo, h.hi, h.d, h.p, sc.c0, S.m, S.gbeg, S.slot_id, sc.P, S.selo,
                  S.go, L.sel, L.G, S.k, hss ? sc.Svec : nullptr, hss ? sc.S_off : nullptr, S.ks,
                  h.tol, h.f, dsw, dsw + 1, 0};
        ia.dlw = (dl && !sc.rowside) ? 1 : 0;
        ia.pd = pd;
        ia.pdat = h.Ap;
        ia.taylor_g = h.taylor_g;
        IdArgs ir = ia;  // the register form writes G^T, and G
        ir.gt_out = 1;
        ir.G_out = L.Gt;
        ir.G2_out = L.G;
        sc.gt_first = all_reg;
        const int wgrid = !h.batched ? 1 : std::min(nl, 2 * dev_cus);
        CsArgs cs{nullptr, nullptr, ldc, lds_cols, std::max(sc.mmax, 1), nullptr, 0, nullptr, 0};
        if (!all_reg) {
          cs.gstride = (int64_t)cs.mmax * ldc + cs.mmax + (int64_t)cw * cw;
          cs.istride = 2 * (int64_t)cs.mmax;
          cs.gscr = tmp.alloc_n<double>((size_t)cs.gstride * wgrid);
          cs.iscr = tmp.alloc_n<int>((size_t)cs.istride * wgrid);
        }
        auto launch_reg = [&](const IdArgs &a, int grid) {
#define SMASH_W_CASE(CM, NTV)                                                    \
  if (cm == CM && nt == NTV) k_compr_w<CM, NTV, lpc, cpg><<<grid, NTV, shw, s>>>(a);
          SMASH_W_CASE(32, 64)
          SMASH_W_CASE(32, 128)
          SMASH_W_CASE(32, 256)
          SMASH_W_CASE(32, 512)
          SMASH_W_CASE(64, 64)
          SMASH_W_CASE(64, 128)
          SMASH_W_CASE(64, 256)
          SMASH_W_CASE(64, 512)
#undef SMASH_W_CASE
          SMASH_CHECK_LAUNCH();
        };
        auto launch_wide = [&](const IdArgs &a, const CsArgs &b, int grid) {
          switch (cw) {
            case 64: k_compr_s<64><<<grid, CS_NT, shs, s>>>(a, b); break;
            case 128: k_compr_s<128><<<grid, CS_NT, shs, s>>>(a, b); break;
            case 224: k_compr_s<224><<<grid, CS_NT, shs, s>>>(a, b); break;
            case 256: k_compr_s<256><<<grid, CS_NT, shs, s>>>(a, b); break;
            default: k_compr_s<512><<<grid, CS_NT, shs, s>>>(a, b); break;
          }
          SMASH_CHECK_LAUNCH();
        };
        // the register QR of k_compr_dq: at most the resident workgroups of
        // the device per launch, and the groups' exchange areas
        const int dq_rc = cw <= 224 ? 64 : 48;  // (RC of k_compr_dq)
        const size_t shd = sizeof(double) * ((size_t)CS_NG * h.d * h.p + (size_t)dq_rc * cw);
        int dq_cap = 0;
        double *dq_slot = nullptr, *dq_R = nullptr, *dq_I = nullptr;
        DqMeta *dq_meta = nullptr;
        int *dq_gc = nullptr;
        unsigned *dq_cnt = nullptr;
        auto dq_kernel = [&]() -> const void * {
          switch (cw) {
            case 64: return (const void *)k_compr_dq<64>;
            case 128: return (const void *)k_compr_dq<128>;
            case 224: return (const void *)k_compr_dq<224>;
            case 256: return (const void *)k_compr_dq<256>;
            default: return nullptr;
          }
        };
        if (h.batched && !all_reg && dq_kernel()) {
          int per_cu = 0;
          if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dq_kernel(), CS_NT, shd) ==
                  hipSuccess &&
              per_cu > 0 && per_cu * dev_cus >= 8 * DQ_MAXW) {
            dq_cap = per_cu * dev_cus;
            dq_slot = tmp.alloc_n<double>((size_t)2 * dq_cap * ldc);
            dq_meta = tmp.alloc_n<DqMeta>((size_t)3 * dq_cap);
            dq_R = tmp.alloc_n<double>((size_t)dq_cap * cw * cw);
            dq_I = tmp.alloc_n<double>((size_t)dq_cap * cw * cw);
            dq_gc = tmp.alloc_n<int>((size_t)dq_cap);
            dq_cnt = tmp.alloc_n<unsigned>((size_t)dq_cap);
          } else {
            (void)hipGetLastError();
          }
        }
        auto launch_dq = [&](const IdArgs &a, const DqArgs &b, int grid) {
          IdArgs a1 = a;
          DqArgs b1 = b;
          void *args[] = {&a1, &b1};
          launch_dq_chained(h.device, dq_kernel(), grid, CS_NT, args, shd, s);
        };
        PhaseTimer pt(h, SMASH_PHASE_COMPR, s);
        if (h.batched) {
          if (all_reg) {
            launch_reg(ir, nl < 8 * dev_cus ? nl : 8 * dev_cus);
          } else {
            // order: the wide form's grids by decreasing size, then the rest
            uint64_t *keys = tmp.alloc_n<uint64_t>(nl), *kalt = tmp.alloc_n<uint64_t>(nl);
            int *vals = tmp.alloc_n<int>(nl), *valt = tmp.alloc_n<int>(nl);
            int *big = tmp.alloc_n<int>(1);
            SMASH_HIP(hipMemsetAsync(big, 0, sizeof(int), s));
            k_order_keys<<<ceil_div(nl, 256), 256, 0, s>>>(nb, ne, S.m, reg_ok ? 256 : -1, keys,
                                                         vals, big);
            SMASH_CHECK_LAUNCH();
            radix_sort_u64(keys, vals, kalt, valt, nl, 17, s, tmp);
            cs.order = vals;
            cs.cnt = big;
            if (cw <= 256 && dq_cap > 0) {
              // the strong RRQR with the columns in registers (grids of up to
              // 2048 points, split over 1-16 workgroups by size); larger
              // grids take the streaming form
              int *exsv = tmp.alloc_n<int>((size_t)L.sel_n);
              int *rng = tmp.alloc_n<int>(12);
              k_dq_ranges<<<1, 64, 0, s>>>(vals, big, S.m, rng);
              SMASH_CHECK_LAUNCH();
              CsArgs c0 = cs;
              c0.first = rng;
              c0.cnt = rng + 1;
              // (grids above DQ_MAXW * DQ_CPW points: none when the level's
              // largest grid is at most that)
              if (sc.mmax > DQ_MAXW * DQ_CPW) launch_wide(ia, c0, wgrid);
              DqArgs da{vals, nullptr, 0, ldc, exsv, dq_slot, dq_meta, dq_R, dq_I, cw * cw,
                        dq_gc, dq_cnt, (int64_t)200000000};
              for (int q = 1; q <= 5; q++) {
                da.nw = DQ_MAXW >> (q - 1);
                da.range = rng + 2 * q;
                const int ngrp = 8 * (dq_cap / (8 * da.nw));
                SMASH_HIP(hipMemsetAsync(dq_cnt, 0, sizeof(unsigned) * ngrp, s));
                launch_dq(ia, da, ngrp * da.nw);
              }
            } else {
              launch_wide(ia, cs, wgrid);
            }
            if (reg_ok) {
              ir.order = vals;
              ir.ord_lo = big;
              launch_reg(ir, nl < 8 * dev_cus ? nl : 8 * dev_cus);
            }
          }
        } else {
          // the plain per-node form: the same choice per node
          std::vector<int> mh((size_t)nl);
          SMASH_HIP(hipMemcpyAsync(mh.data(), S.m + nb, sizeof(int) * nl, hipMemcpyDeviceToHost,
                                   s));
          SMASH_HIP(hipStreamSynchronize(s));
          int *one = nullptr;
          if (!all_reg) {
            one = tmp.alloc_n<int>(1);
            SMASH_HIP(hipMemsetD32Async((hipDeviceptr_t)one, 1, 1, s));
          }
          cs.cnt = one;
          for (int i = nb; i < ne; i++) {
            IdArgs a1 = (reg_ok && mh[i - nb] <= 256) ? ir : ia;
            a1.nb = i;
            a1.ne = i + 1;
            if (hss) a1.S_off = sc.S_off + (i - nb);
            if (reg_ok && mh[i - nb] <= 256)
              launch_reg(a1, 1);
            else
              launch_wide(a1, cs, 1);
          }
        }
      }
      // the other orientation of G (the up pass reads G, the down pass G^T)
      for (auto &sc : sides) {
        Side &S = *sc.S;
        LevelSide &L = S.lv[l];
        if (sc.gt_first) continue;  // the register kernel wrote both
        k_transpose_G<<<nl, 256, 0, s>>>(nb, ne, S.m, S.k, S.go, L.G, L.Gt);
        SMASH_CHECK_LAUNCH();
      }
      // (d) skeleton slots of this level (capacity reserved up front)
      for (size_t q = 0; q < sides.size(); q++) {
        SideCtx &sc = sides[q];
        Side &S = *sc.S;
        if (nl <= LV_NT * LV_PER) {
          k_level_slots1<<<1, LV_NT, 0, s>>>(nb, ne, S.k, S.hbeg, dslots + q);
          SMASH_CHECK_LAUNCH();
        } else {
          int64_t *ck = tmp.alloc_n<int64_t>(nl), *ok = tmp.alloc_n<int64_t>(nl + 1);
          k_kcopy<<<ceil_div(nl, 256), 256, 0, s>>>(nb, ne, S.k, ck);
          SMASH_CHECK_LAUNCH();
          scan_i64(ck, ok, nl, dslots + q, s, tmp);
          copy_i64(dslots + q, ok + nl, s);
          k_set_hbeg<<<ceil_div(nl, 256), 256, 0, s>>>(nb, ne, ok, S.hbeg);
          SMASH_CHECK_LAUNCH();
        }
        {
          PhaseTimer pt(h, SMASH_PHASE_SLOTS, s);
          k_slot_ids<<<nl, 64, 0, s>>>(nb, ne, S.k, S.hbeg, S.gbeg, S.selo, S.lv[l].sel,
                                       S.slot_id);
          SMASH_CHECK_LAUNCH();
        }
      }
      // per-level temporaries are dropped once they grow large (the swap
      // counters and the max cells live in `keep`, allocated once)
      if (tmp.bytes > ((int64_t)256 << 20)) {
        SMASH_HIP(hipStreamSynchronize(s));
        tmp.release();
      }
    }
    int herr[2] = {0, 0};
    {
      // the coupling blocks' sizes and offsets (their total comes with the
      // same host read)
      coupling_offsets(h, tmp);
      const int64_t *pin = pick_words(s, {{dsw, 4},
                                          {dsw + 1, 4},
                                          {dslots, 8},
                                          {dslots + 1, 8},
                                          {dsw + 2, 4},
                                          {h.boff + h.nL, 8}});
      herr[0] = (int)pin[0];
      herr[1] = (int)pin[1];
      for (size_t q = 0; q < sides.size(); q++) sides[q].S->nslots = pin[2 + q];
      h.nleaves = (int)pin[4];
      h.b_entries = pin[5];
    }
    if (herr[1] & 2)
      throw Error{SMASH_E_DEVICE, "compr: the workgroups of a node did not meet in time"};
    if (herr[1]) throw Error{SMASH_E_NUMERIC, "strong RRQR swap cap reached"};
    h.total_swaps = herr[0];
    // apply copies
    if (h.apply_prec == SMASH_F32) {
      for (auto &sc : sides) {
        for (int l = 2; l <= h.nlevels; l++) {
          LevelSide &L = sc.S->lv[l];
          L.G32 = h.mem.alloc_n<float>(L.g_n);
          L.Gt32 = h.mem.alloc_n<float>(L.g_n);
          if (L.g_n > 0) {
            k_to_f32<<<ceil_div(L.g_n, 256), 256, 0, s>>>(L.G, L.G32, L.g_n);
            SMASH_CHECK_LAUNCH();
            k_to_f32<<<ceil_div(L.g_n, 256), 256, 0, s>>>(L.Gt, L.Gt32, L.g_n);
            SMASH_CHECK_LAUNCH();
          }
        }
      }
    }
    if (h.apply_prec == SMASH_BF16) {
      for (auto &sc : sides) {
        Side &S = *sc.S;
        S.gobu = h.mem.alloc_n<int64_t>(h.nnodes);
        S.gobd = h.mem.alloc_n<int64_t>(h.nnodes);
        for (int l = 2; l <= h.nlevels; l++) {
          const int nb = h.level_beg[l - 1], ne = h.level_beg[l], nl = ne - nb;
          LevelSide &L = S.lv[l];
          int64_t *cu = tmp.alloc_n<int64_t>(nl), *cd = tmp.alloc_n<int64_t>(nl);
          int64_t *ou = tmp.alloc_n<int64_t>(nl + 1), *od = tmp.alloc_n<int64_t>(nl + 1);
          k_gb_sizes<<<ceil_div(nl, 256), 256, 0, s>>>(nb, ne, S.m, S.k, cu, cd);
          SMASH_CHECK_LAUNCH();
          scan_i64(cu, ou, nl, nullptr, s, tmp);
          scan_i64(cd, od, nl, nullptr, s, tmp);
          k_set_rel<<<ceil_div(nl, 256), 256, 0, s>>>(nb, ne, ou, S.gobu);
          SMASH_CHECK_LAUNCH();
          k_set_rel<<<ceil_div(nl, 256), 256, 0, s>>>(nb, ne, od, S.gobd);
          SMASH_CHECK_LAUNCH();
          const int64_t *pin = pick_words(s, {{ou + nl, 8}, {od + nl, 8}});
          const int64_t tot[2] = {pin[0], pin[1]};
          L.gbu_n = tot[0];
          L.gbd_n = tot[1];
          L.Gbu = h.mem.alloc_n<unsigned short>(tot[0]);
          L.Gbd = h.mem.alloc_n<unsigned short>(tot[1]);
          k_g_to_bf16<<<nl, 256, 0, s>>>(nb, ne, S.m, S.k, S.go, L.G, S.gobu, S.gobd, L.Gbu,
                                         L.Gbd);
          SMASH_CHECK_LAUNCH();
        }
      }
    }
    defer_release(h, tmp);
    defer_release(h, keep);
  } catch (...) {
    (void)hipStreamSynchronize(s);
    tmp.release();
    keep.release();
    throw;
  }
}

}  // namespace smash
