// blocks.hip -- coupling blocks B_ij = A|(i-hat x j-hat) over the admissible
// leaves L (eqs. (3.15), (3.19)) and near-field blocks A|(i x j) over the
// inadmissible leaves L^- (eqs. (3.15), (3.20)), evaluated from the kernel
// and stored in the apply precision.  Each block is stored column-major
// (row index fastest) so that the product reads it with unit stride.
#include "common.cuh"

namespace smash {

// entries per block; pad8: columns rounded up to a multiple of 8 (the BF16
// matrix-core operand order)
__global__ void k_block_sizes(int64_t n, const int *pi, const int *pj, const int *ki,
                              const int *kj, int pad8, int64_t *cnt) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const int c = kj[pj[a]];
  cnt[a] = (int64_t)ki[pi[a]] * (pad8 ? (c + 7) & ~7 : c);
}

__global__ void k_near_sizes(int64_t n, const int *pi, const int *pj, const int *xb,
                             const int *xe, const int *yb, const int *ye, int pad8,
                             int64_t *cnt) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const int c = ye[pj[a]] - yb[pj[a]];
  cnt[a] = (int64_t)(xe[pi[a]] - xb[pi[a]]) * (pad8 ? (c + 7) & ~7 : c);
}

struct EvalArgs {
  int64_t npairs;
  const int *pi, *pj;
  const int64_t *off;
  // row points of block e: Xp[rid[rbeg[i] + a]] (rid == null: Xp[rbeg[i] + a])
  const int64_t *rbeg;
  const int *rbeg32;
  const int *rcnt_k;  // rows per node (k or point count via rend32)
  const int *rend32;
  const int *rid;
  const int64_t *cbeg;
  const int *cbeg32;
  const int *ccnt_k;
  const int *cend32;
  const int *cid;
  const double *Xp, *Yp;
  int d, kid;
  double diag;
  const double *pd;  // double-layer kernel: per-point data by point id (X = Y)
};

// Coordinates of a block's rows and columns are staged in LDS (up to
// EV_STAGE points each), and every thread walks its entries with a running
// (row, column) pair instead of dividing by the row count per entry.
constexpr int EV_STAGE = 256;

template <class T, bool F32MATH, int KID, int D>
__global__ void __launch_bounds__(256) k_eval_blocks(EvalArgs A, T *out) {
  __shared__ double xs[EV_STAGE * 3], ys[EV_STAGE * 3];
  constexpr int d = D;
  for (int64_t e = blockIdx.x; e < A.npairs; e += gridDim.x) {
    int i = A.pi[e], j = A.pj[e];
    int64_t r0, c0;
    int nr, nc;
    if (A.rbeg) {
      r0 = A.rbeg[i];
      nr = A.rcnt_k[i];
    } else {
      r0 = A.rbeg32[i];
      nr = A.rend32[i] - A.rbeg32[i];
    }
    if (A.cbeg) {
      c0 = A.cbeg[j];
      nc = A.ccnt_k[j];
    } else {
      c0 = A.cbeg32[j];
      nc = A.cend32[j] - A.cbeg32[j];
    }
    T *B = out + A.off[e];
    const int tot = nr * nc;
    if (tot == 0) continue;
    // (the double-layer kernel also needs each point's data: not staged)
    const bool staged = KID != SMASH_KERNEL_DOUBLE_LAYER && nr <= EV_STAGE && nc <= EV_STAGE;
    __syncthreads();  // the previous pair's readers are done with xs / ys
    if (staged) {
      for (int q = threadIdx.x; q < nr * d; q += blockDim.x) {
        const int a = q / d, t = q - a * d;
        const int64_t xr = A.rid ? A.rid[r0 + a] : r0 + a;
        xs[q] = A.Xp[xr * d + t];
      }
      for (int q = threadIdx.x; q < nc * d; q += blockDim.x) {
        const int b = q / d, t = q - b * d;
        const int64_t yc = A.cid ? A.cid[c0 + b] : c0 + b;
        ys[q] = A.Yp[yc * d + t];
      }
    }
    __syncthreads();
    // column-major: row fastest; (a, b) of entry q advanced by the stride
    const int st = blockDim.x, sb = st / nr, sa = st - sb * nr;
    int b = threadIdx.x / nr, a = threadIdx.x - b * nr;
    for (int q = threadIdx.x; q < tot; q += st) {
      const double *xp, *yp, *ax = nullptr, *ay = nullptr;
      if (staged) {
        xp = xs + a * d;
        yp = ys + b * d;
      } else {
        const int64_t xr = A.rid ? A.rid[r0 + a] : r0 + a;
        const int64_t yc = A.cid ? A.cid[c0 + b] : c0 + b;
        xp = A.Xp + xr * d;
        yp = A.Yp + yc * d;
        if (KID == SMASH_KERNEL_DOUBLE_LAYER) {
          ax = A.pd + 3 * xr;
          ay = A.pd + 3 * yc;
        }
      }
      if (F32MATH)
        B[q] = (T)kernel_f32_t<KID, D>(xp, yp, (float)A.diag, ax, ay);
      else
        B[q] = (T)kernel_f64_t<KID, D>(xp, yp, A.diag, ax, ay);
      a += sa;
      b += sb;
      if (a >= nr) {
        a -= nr;
        b++;
      }
    }
  }
}

// BF16 blocks in the matrix-core operand order: entry (a, b) of an nr x nc
// block at ((b/8) * nr + a) * 8 + b%8, columns padded with zeros to a
// multiple of 8, so eight consecutive columns of one row are one 16-byte load.
template <bool F32MATH>
__global__ void __launch_bounds__(256) k_eval_blocks_bf16(EvalArgs A, unsigned short *out) {
  for (int64_t e = blockIdx.x; e < A.npairs; e += gridDim.x) {
    int i = A.pi[e], j = A.pj[e];
    int64_t r0, c0;
    int nr, nc;
    if (A.rbeg) {
      r0 = A.rbeg[i];
      nr = A.rcnt_k[i];
    } else {
      r0 = A.rbeg32[i];
      nr = A.rend32[i] - A.rbeg32[i];
    }
    if (A.cbeg) {
      c0 = A.cbeg[j];
      nc = A.ccnt_k[j];
    } else {
      c0 = A.cbeg32[j];
      nc = A.cend32[j] - A.cbeg32[j];
    }
    unsigned short *B = out + A.off[e];
    const int tot = nr * ((nc + 7) & ~7);
    for (int q = threadIdx.x; q < tot; q += blockDim.x) {
      const int b8 = q / (nr * 8), r = q - b8 * nr * 8, a = r >> 3, b = b8 * 8 + (r & 7);
      float v = 0.0f;
      if (b < nc) {
        int64_t xr = A.rid ? A.rid[r0 + a] : r0 + a;
        int64_t yc = A.cid ? A.cid[c0 + b] : c0 + b;
        const double *xp = A.Xp + xr * A.d, *yp = A.Yp + yc * A.d;
        const double *ax = A.pd ? A.pd + 3 * xr : nullptr, *ay = A.pd ? A.pd + 3 * yc : nullptr;
        v = F32MATH ? kernel_f32(A.kid, xp, yp, A.d, (float)A.diag, ax, ay)
                    : (float)kernel_f64(A.kid, xp, yp, A.d, A.diag, ax, ay);
      }
      B[q] = bf16_bits(v);
    }
  }
}

static void eval_launch_bf16(EvalArgs &ea, unsigned short *out, bool f32math, hipStream_t s) {
  int nblk = ea.npairs < (1 << 20) ? (int)ea.npairs : (1 << 20);
  if (nblk <= 0) return;
  if (f32math)
    k_eval_blocks_bf16<true><<<nblk, 256, 0, s>>>(ea, out);
  else
    k_eval_blocks_bf16<false><<<nblk, 256, 0, s>>>(ea, out);
  SMASH_CHECK_LAUNCH();
}

template <class T, bool F32MATH, int KID>
static void eval_launch_k(int nblk, EvalArgs &ea, T *out, hipStream_t s) {
  switch (ea.d) {
    case 1: k_eval_blocks<T, F32MATH, KID, 1><<<nblk, 256, 0, s>>>(ea, out); break;
    case 2: k_eval_blocks<T, F32MATH, KID, 2><<<nblk, 256, 0, s>>>(ea, out); break;
    default: k_eval_blocks<T, F32MATH, KID, 3><<<nblk, 256, 0, s>>>(ea, out); break;
  }
}

template <class T, bool F32MATH>
static void eval_launch_m(int nblk, EvalArgs &ea, T *out, hipStream_t s) {
  switch (ea.kid) {
    case SMASH_KERNEL_INV_R: eval_launch_k<T, F32MATH, SMASH_KERNEL_INV_R>(nblk, ea, out, s); break;
    case SMASH_KERNEL_LOG_R: eval_launch_k<T, F32MATH, SMASH_KERNEL_LOG_R>(nblk, ea, out, s); break;
    case SMASH_KERNEL_EXP_R: eval_launch_k<T, F32MATH, SMASH_KERNEL_EXP_R>(nblk, ea, out, s); break;
    case SMASH_KERNEL_DOUBLE_LAYER:  // dim 2 only
      k_eval_blocks<T, F32MATH, SMASH_KERNEL_DOUBLE_LAYER, 2><<<nblk, 256, 0, s>>>(ea, out);
      break;
    default: eval_launch_k<T, F32MATH, SMASH_KERNEL_CAUCHY>(nblk, ea, out, s); break;
  }
}

template <class T>
static void eval_launch(EvalArgs &ea, T *out, bool f32math, hipStream_t s) {
  int nblk = ea.npairs < (1 << 20) ? (int)ea.npairs : (1 << 20);
  if (nblk <= 0) return;
  if (f32math)
    eval_launch_m<T, true>(nblk, ea, out, s);
  else
    eval_launch_m<T, false>(nblk, ea, out, s);
  SMASH_CHECK_LAUNCH();
}

// the coupling pairs [p0, p1): rows at the row side's skeleton slots,
// columns at the column side's
static EvalArgs coupling_args(Handle &h, int64_t p0, int64_t p1) {
  Side &R = h.row, &C = *h.col;
  EvalArgs ea{};
  ea.d = h.d;
  ea.kid = h.kid;
  ea.diag = h.diag;
  ea.Xp = h.Xp;
  ea.Yp = h.Yp;
  ea.npairs = p1 - p0;
  ea.pi = h.Li + p0;
  ea.pj = h.Lj + p0;
  ea.off = h.boff + p0;
  ea.rbeg = R.hbeg;
  ea.rcnt_k = R.k;
  ea.rid = R.slot_id;
  ea.cbeg = C.hbeg;
  ea.ccnt_k = C.k;
  ea.cid = C.slot_id;
  ea.pd = h.Ap;
  return ea;
}

void eval_coupling_range(Handle &h, int64_t p0, int64_t p1, void *base, hipStream_t s) {
  if (p1 <= p0) return;
  EvalArgs ea = coupling_args(h, p0, p1);
  const bool f32math = h.eval_prec == SMASH_F32;
  if (h.apply_prec == SMASH_F64)
    eval_launch(ea, (double *)base, f32math, s);
  else if (h.apply_prec == SMASH_BF16)
    eval_launch_bf16(ea, (unsigned short *)base, f32math, s);
  else
    eval_launch(ea, (float *)base, f32math, s);
}

// Chunk boundaries of the evaluated coupling form: boundary c (< nch) is
// the first row node whose pairs start at or past entry c * cap; the last
// one is nnodes.  Also the first pair and entry of each chunk.
__global__ void k_chunk_bounds(int nnodes, const int *Lrow, const int64_t *boff, int64_t cap,
                               int nch, int *node, int64_t *pair, int64_t *ent) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > nch) return;
  int lo = 0, hi = nnodes;
  if (c == nch) {
    lo = nnodes;
  } else {
    const int64_t target = (int64_t)c * cap;
    while (lo < hi) {
      const int mid = lo + (hi - lo) / 2;
      if (boff[Lrow[mid]] >= target)
        hi = mid;
      else
        lo = mid + 1;
    }
  }
  node[c] = lo;
  pair[c] = Lrow[lo];
  ent[c] = boff[Lrow[lo]];
}

// Coordinates of every slot of one side: out[s d + t] = P[slot_id[s] d + t].
__global__ void k_slot_coords(int64_t nslots, int d, const int *slot_id, const double *P,
                              double *out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nslots * d) return;
  const int64_t sl = e / d;
  out[e] = P[(int64_t)slot_id[sl] * d + (e - sl * d)];
}

// One second stream and completion event per device and host thread,
// default priority, created on first use and kept for the process.
static void side_stream(int dev, hipStream_t &st, hipEvent_t &ready, hipEvent_t &done) {
  struct Side3 {
    hipStream_t s = nullptr;
    hipEvent_t r = nullptr, d = nullptr;
  };
  thread_local std::vector<Side3> v;
  if ((int)v.size() <= dev) v.resize(dev + 1);
  Side3 &x = v[dev];
  if (!x.s) {
    SMASH_HIP(hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking));
    SMASH_HIP(hipEventCreateWithFlags(&x.r, hipEventDisableTiming));
    SMASH_HIP(hipEventCreateWithFlags(&x.d, hipEventDisableTiming));
  }
  st = x.s;
  ready = x.r;
  done = x.d;
}

// Near-field blocks (eqs. (3.15), (3.20)): they need only the tree and L^-,
// so they are evaluated on a second stream while the generators are built
// (whose upper levels occupy few compute units).  near_offsets scans their
// sizes; near_launch allocates them (given their total) and starts the
// evaluation.
void near_offsets(Handle &h) {
  hipStream_t s = h.stream;
  DeviceArena tmp;
  tmp.stream = s;
  try {
    const bool bf = h.apply_prec == SMASH_BF16;
    int64_t *ncnt = tmp.alloc_n<int64_t>(h.nLm);
    h.nboff = h.mem.alloc_n<int64_t>(h.nLm + 1);
    if (h.nLm > 0) {
      k_near_sizes<<<ceil_div(h.nLm, 256), 256, 0, s>>>(h.nLm, h.Lmi, h.Lmj, h.xb, h.xe, h.yb,
                                                        h.ye, bf ? 1 : 0, ncnt);
      SMASH_CHECK_LAUNCH();
    }
    scan_i64(ncnt, h.nboff, h.nLm, nullptr, s, tmp);
    int dev = 0;
    SMASH_HIP(hipGetDevice(&dev));
    hipEvent_t ready;
    side_stream(dev, h.side, ready, h.side_done);
    defer_release(h, tmp);
  } catch (...) {
    (void)hipStreamSynchronize(s);
    tmp.release();
    throw;
  }
}

void near_launch(Handle &h, int64_t n_entries) {
  hipStream_t s = h.stream;
  const bool bf = h.apply_prec == SMASH_BF16;
  size_t es = h.apply_prec == SMASH_F64 ? sizeof(double)
              : bf                      ? sizeof(unsigned short)
                                        : sizeof(float);
  bool f32math = h.eval_prec == SMASH_F32;
  h.n_entries = n_entries;
  h.Bn = h.mem.alloc(es * (size_t)(h.n_entries > 0 ? h.n_entries : 1));
  int dev = 0;
  SMASH_HIP(hipGetDevice(&dev));
  hipEvent_t ready;
  side_stream(dev, h.side, ready, h.side_done);
  // everything above (the lists, offsets and Bn) is ordered before the side work
  SMASH_HIP(hipEventRecord(ready, s));
  SMASH_HIP(hipStreamWaitEvent(h.side, ready, 0));
  EvalArgs en{};
  en.d = h.d;
  en.kid = h.kid;
  en.diag = h.diag;
  en.Xp = h.Xp;
  en.Yp = h.Yp;
  en.npairs = h.nLm;
  en.pi = h.Lmi;
  en.pj = h.Lmj;
  en.off = h.nboff;
  en.rbeg32 = h.xb;
  en.rend32 = h.xe;
  en.cbeg32 = h.yb;
  en.cend32 = h.ye;
  en.pd = h.Ap;
  {
    PhaseTimer pt(h, SMASH_PHASE_BLOCKS, h.side);
    if (h.apply_prec == SMASH_F64)
      eval_launch(en, (double *)h.Bn, f32math, h.side);
    else if (bf)
      eval_launch_bf16(en, (unsigned short *)h.Bn, f32math, h.side);
    else
      eval_launch(en, (float *)h.Bn, f32math, h.side);
  }
  SMASH_HIP(hipEventRecord(h.side_done, h.side));
}

void coupling_offsets(Handle &h, DeviceArena &tmp) {
  hipStream_t s = h.stream;
  int64_t *cnt = tmp.alloc_n<int64_t>(h.nL);
  h.boff = h.mem.alloc_n<int64_t>(h.nL + 1);
  if (h.nL > 0) {
    k_block_sizes<<<ceil_div(h.nL, 256), 256, 0, s>>>(h.nL, h.Li, h.Lj, h.row.k, h.col->k,
                                                      h.apply_prec == SMASH_BF16 ? 1 : 0, cnt);
    SMASH_CHECK_LAUNCH();
  }
  scan_i64(cnt, h.boff, h.nL, nullptr, s, tmp);
}

void build_blocks(Handle &h) {
  hipStream_t s = h.stream;
  DeviceArena tmp;
  tmp.stream = s;
  try {
    Side &R = h.row, &C = *h.col;
    const bool bf = h.apply_prec == SMASH_BF16;
    size_t es = h.apply_prec == SMASH_F64 ? sizeof(double)
                : bf                      ? sizeof(unsigned short)
                                          : sizeof(float);
    bool f32math = h.eval_prec == SMASH_F32;
    (void)f32math;
    // coupling: offsets and total were set with the generators' last host
    // read (coupling_offsets)
    // coupling blocks stored, or evaluated by each product in chunks
    bool evaluated = h.coupling_mode == SMASH_COUPLING_EVALUATED;
    if (h.coupling_mode == SMASH_COUPLING_AUTO) {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess)
        evaluated = (double)es * (double)h.b_entries > 0.75 * (double)fr;
    }
    h.coupling_eval = evaluated && h.nL > 0 && h.b_entries > 0;
    // FP64 and FP32 apply: the blocks are evaluated inside the contraction
    // from the skeleton slots' coordinates; BF16 apply: a chunk of pairs at
    // a time into a workspace, then the BF16 contraction
    h.coupling_fused = h.coupling_eval && !bf;
    if (h.coupling_fused) {
      auto coords = [&](Side &S, const double *P) {
        double *c = h.mem.alloc_n<double>((size_t)S.nslots * h.d);
        if (S.nslots > 0) {
          k_slot_coords<<<ceil_div(S.nslots * h.d, 256), 256, 0, s>>>(S.nslots, h.d, S.slot_id,
                                                                      P, c);
          SMASH_CHECK_LAUNCH();
        }
        return c;
      };
      h.xs_slot = coords(R, h.Xp);
      h.ys_slot = h.col == &h.row && h.Yp == h.Xp ? h.xs_slot : coords(C, h.Yp);
      h.B = nullptr;
    } else if (h.coupling_eval) {
      const int64_t cap = h.coupling_chunk > 0
                              ? h.coupling_chunk
                              : std::max<int64_t>((int64_t)(256 << 20) / (int64_t)es, 1);
      const int nch = (int)((h.b_entries + cap - 1) / cap);
      int *dn = tmp.alloc_n<int>(nch + 1);
      int64_t *dp = tmp.alloc_n<int64_t>(nch + 1), *de = tmp.alloc_n<int64_t>(nch + 1);
      k_chunk_bounds<<<ceil_div(nch + 1, 256), 256, 0, s>>>((int)h.nnodes, h.Lrow, h.boff, cap,
                                                           nch, dn, dp, de);
      SMASH_CHECK_LAUNCH();
      h.cchunk_node.assign(nch + 1, 0);
      h.cchunk_pair.assign(nch + 1, 0);
      h.cchunk_ent.assign(nch + 1, 0);
      SMASH_HIP(hipMemcpyAsync(h.cchunk_node.data(), dn, sizeof(int) * (nch + 1),
                               hipMemcpyDeviceToHost, s));
      SMASH_HIP(hipMemcpyAsync(h.cchunk_pair.data(), dp, sizeof(int64_t) * (nch + 1),
                               hipMemcpyDeviceToHost, s));
      SMASH_HIP(hipMemcpyAsync(h.cchunk_ent.data(), de, sizeof(int64_t) * (nch + 1),
                               hipMemcpyDeviceToHost, s));
      SMASH_HIP(hipStreamSynchronize(s));  // (pageable destinations)
      h.bws_entries = 1;
      for (int c = 0; c < nch; c++)
        h.bws_entries = std::max(h.bws_entries, h.cchunk_ent[c + 1] - h.cchunk_ent[c]);
      h.Bws = h.mem.alloc(es * (size_t)h.bws_entries);
      h.B = nullptr;
    } else {
      h.B = h.mem.alloc(es * (size_t)(h.b_entries > 0 ? h.b_entries : 1));
    }
    PhaseTimer pt(h, SMASH_PHASE_BLOCKS, s);
    // B_ij = A(X at i-hat, Y at j-hat): skeleton slots of both sides
    if (!h.coupling_eval) eval_coupling_range(h, 0, h.nL, h.B, s);
    // the near-field blocks of the second stream complete before the build ends
    if (h.side) SMASH_HIP(hipStreamWaitEvent(s, h.side_done, 0));
    SMASH_HIP(hipStreamSynchronize(s));
    tmp.release();
  } catch (...) {
    (void)hipStreamSynchronize(s);
    if (h.side) (void)hipStreamSynchronize(h.side);
    tmp.release();
    throw;
  }
}

}  // namespace smash
