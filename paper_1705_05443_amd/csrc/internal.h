// internal.h -- shared declarations of libsmash (not part of the ABI).
//
// Device data layout (all row-major):
//  * Points are kept permuted: Xp (nx x d) and Yp (ny x d) FP64, in the
//    depth-first order of the partition tree, so every node owns a
//    contiguous range [xb, xe) of X and [yb, ye) of Y.
//  * Nodes are numbered level by level (root = node 0, level 1), Morton
//    order inside a level; the children of a node are consecutive.
//  * Slot space (one per side): slots [0, n) are the permuted points; then
//    each level l = L, L-1, ..., 2 appends one slot per skeleton point of its
//    nodes.  A node's current grid (eqs. (3.6), (3.14), (3.18)) is the slot
//    range [gbeg, gbeg + m) -- a leaf's own points, or the consecutive
//    skeleton slots of its children -- and its skeleton occupies
//    [hbeg, hbeg + k).  slot_id maps a slot to its permuted point id.
//    The product uses the same slot space for q / q-hat (column side) and
//    z / z-hat (row side).
//  * Per node and side: sel (m int32: skeleton positions ascending, then the
//    remaining positions ascending) and G ((m-k) x k), the interpolative
//    decomposition U = P [I; G] of eq. (2.11), stored per level.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <cstring>
#include <atomic>
#include <initializer_list>
#include <utility>
#include <vector>

#include "../../include/smash.h"

namespace smash {

// ---------------------------------------------------------------- errors
struct Error {
  int code;
  std::string msg;
};

#define SMASH_HIP(call)                                                          \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      throw ::smash::Error{SMASH_E_DEVICE, std::string(#call) + ": " +           \
                                               hipGetErrorString(e_)};           \
  } while (0)

#define SMASH_CHECK_LAUNCH() SMASH_HIP(hipGetLastError())

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------- allocator
// Bump allocation (256-byte aligned) inside chunks taken stream-ordered from
// the device's default memory pool (kept cached across builds), so a build
// makes a handful of pool calls instead of one per array.  release() returns
// every chunk.
// Caller's allocator hooks of a handle (smash_options.alloc/.free).
struct AllocHooks {
  smash_alloc_fn alloc = nullptr;
  smash_free_fn free = nullptr;
  void *ctx = nullptr;
};
// The hooks of the handle whose call runs on this host thread (null: the
// library's pool).  An arena takes them at its first allocation and keeps
// them for its release.
const AllocHooks *current_hooks();
struct HooksScope {
  const AllocHooks *prev;
  explicit HooksScope(const AllocHooks *h);
  ~HooksScope();
};

// Device bytes held by a construction's arenas (chunks, whatever their
// source): live now and the most at any time.  An arena takes the account of
// the construction running on its host thread at its first allocation.
struct MemAcct {
  std::atomic<int64_t> live{0}, peak{0};
  void add(int64_t b) {
    const int64_t v = live.fetch_add(b) + b;
    int64_t p = peak.load();
    while (v > p && !peak.compare_exchange_weak(p, v)) {
    }
  }
};
MemAcct *current_acct();
struct AcctScope {
  MemAcct *prev;
  explicit AcctScope(MemAcct *a);
  ~AcctScope();
};

// Frees the idle cached chunks of device `dev`.
void trim_chunk_cache(int dev);

struct DeviceArena {
  hipStream_t stream = nullptr;
  const AllocHooks *hooks = nullptr;  // set at the first allocation
  MemAcct *acct = nullptr;            // set at the first allocation
  bool bound = false;
  std::vector<std::pair<void *, size_t>> blocks;  // (base, size) of each chunk
  char *cur = nullptr;
  size_t left = 0;
  size_t chunk = (size_t)32 << 20;
  int64_t bytes = 0;  // bytes handed out
  void *alloc(size_t n);
  template <class T>
  T *alloc_n(size_t n) {
    return (T *)alloc(sizeof(T) * (n ? n : 1));
  }
  // Gives the chunks back.  idle = true: no queued work uses them any more
  // (the caller synchronized their stream), so they go to the process-wide
  // chunk cache for the next arena; otherwise hipFreeAsync on `stream`.
  void release(bool idle = true);
};

// ---------------------------------------------------------------- scans / sort
// Exclusive scan of int64 values: out[i] = base + sum_{j<i} in[i]; out[n] =
// base + total (out has n+1 entries).  base_dev may be null (then 0).
void scan_i64(const int64_t *in, int64_t *out, int64_t n, const int64_t *base_dev,
              hipStream_t s, DeviceArena &tmp);
// Stable LSD radix sort of (key, value) pairs on bits [0, nbits).  Results
// land in keys/vals (alt buffers are scratch of the same size).
// stable LSD sort by key bits [lo_bit, nbits) (4 bits per pass)
void radix_sort_u64(uint64_t *keys, int32_t *vals, uint64_t *keys_alt, int32_t *vals_alt,
                    int64_t n, int nbits, hipStream_t s, DeviceArena &tmp, int lo_bit = 0);

// ---------------------------------------------------------------- host reads
// A per-thread pinned buffer of 64 words (hipHostMalloc, kept for the life of
// the thread) for the build's small device-to-host reads: the copies go
// straight to pinned memory and one stream synchronization covers them.
int64_t *pinned_words();
// Waits until `s` has passed everything enqueued so far by polling an event
// (a host readback in the build waits for a short tail of small kernels;
// polling wakes sooner than a blocking synchronisation)
void stream_wait(hipStream_t s);
// Copies up to 16 device words (8-byte, or 4-byte int sign-extended) into
// pinned_words()[0..n) with one tiny kernel that writes host memory
// directly, then waits for `s`.  items: (device pointer, 4 or 8).
int64_t *pick_words(hipStream_t s, std::initializer_list<std::pair<const void *, int>> items);
template <class T>
T read_one(hipStream_t s, const T *dev) {
  int64_t *p = pinned_words();
  SMASH_HIP(hipMemcpyAsync(p, dev, sizeof(T), hipMemcpyDeviceToHost, s));
  stream_wait(s);
  T v;
  std::memcpy(&v, p, sizeof(T));
  return v;
}
// Sets one device int64 from a kernel argument (no host-memory copy).
void set_i64(int64_t *dev, int64_t v, hipStream_t s);
// *dst = *src on the stream (device to device, one value)
void copy_i64(int64_t *dst, const int64_t *src, hipStream_t s);

// ---------------------------------------------------------------- handle
struct LevelSide {
  int *sel = nullptr;     // concatenated sel of the level's nodes
  double *G = nullptr;    // concatenated G, (m-k) x k per node (FP64 master)
  double *Gt = nullptr;   // the same transposed, k x (m-k) per node
  float *G32 = nullptr;   // FP32 apply copies
  float *Gt32 = nullptr;
  // BF16 apply copies in the matrix-core operand order (eight consecutive
  // K entries per 16-byte load): up  = H^T, k x (m-k), K = grid row a,
  // stored [a/8][t][a%8]; down = G, (m-k) x k, K = skeleton index t, stored
  // [t/8][a][t%8]; K padded with zeros to a multiple of 8
  unsigned short *Gbu = nullptr, *Gbd = nullptr;
  int64_t sel_n = 0, g_n = 0, gbu_n = 0, gbd_n = 0;
};

struct Side {
  int *m = nullptr, *k = nullptr, *ks = nullptr;  // per node
  int64_t *gbeg = nullptr, *hbeg = nullptr, *selo = nullptr, *go = nullptr;
  int64_t *gobu = nullptr, *gobd = nullptr;  // BF16 copy offsets per node
  int *slot_id = nullptr;
  int64_t slot_cap = 0, nslots = 0;
  std::vector<LevelSide> lv;  // indexed by level (1-based; [0] unused)
  int64_t sum_k = 0, g_total = 0;
  int max_k = 0;
};

struct GraphEntry {
  const void *X;
  int64_t ldx;
  int nrhs;
  void *Y;
  int64_t ldy;
  int calls;
  hipGraphExec_t exec;
  hipEvent_t done;  // recorded after each launch of exec (nullptr before the first)
};

struct Handle {
  // problem
  int d = 0, kid = 0, adm = 0, leaf = 0, p = 0;
  double tol = 0, tau = 0, eps_svd = 0, f = 2, diag = 0;
  int eval_prec = SMASH_F64, apply_prec = SMASH_F64, batched = 1, mv_split_nodes = 1024;
  int mv_xcd_run = 16;
  int64_t nx = 0, ny = 0;
  double taylor_g = 0.0;  // > 0: Taylor basis (2.4)-(2.5) with this g, else interpolation (2.2)
  bool same_xy = false, reuse = false;
  int device = 0;
  hipStream_t stream = nullptr;
  DeviceArena mem;
  // permuted points
  double *Xp = nullptr, *Yp = nullptr;
  // double-layer kernel: per-point data (m_1, m_2, diagonal), n x 3, as
  // given (pdata_in, borrowed) and permuted with the points (Ap)
  const double *pdata_in = nullptr;
  double *Ap = nullptr;
  int *perm_x = nullptr, *perm_y = nullptr;
  // geometry
  bool has_root = false;
  double root_lo[3] = {0, 0, 0}, root_hi[3] = {0, 0, 0};
  int bpl = 1, max_split = 0;
  // tree
  int nnodes = 0, nlevels = 0, nleaves = 0;
  std::vector<int> level_beg;  // size nlevels+1
  int *level = nullptr, *parent = nullptr, *first_child = nullptr, *nchild = nullptr;
  int *xb = nullptr, *xe = nullptr, *yb = nullptr, *ye = nullptr;
  double *lo = nullptr, *hi = nullptr;  // nnodes x 3
  // pair lists (sorted by (i, j)) and CSR rows
  int64_t nL = 0, nLm = 0;
  int *Li = nullptr, *Lj = nullptr, *Lmi = nullptr, *Lmj = nullptr;
  int *Lrow = nullptr, *Lmrow = nullptr;
  int *Nrow = nullptr, *Ncol = nullptr;  // HSS N_i
  int64_t nN = 0;
  // sides
  Side row, col_own;
  Side *col = nullptr;  // == &row when reused
  // blocks (apply precision)
  int64_t *boff = nullptr, *nboff = nullptr;
  void *B = nullptr, *Bn = nullptr;
  int64_t b_entries = 0, n_entries = 0;
  // the near-field blocks are evaluated on a second stream (same priority)
  // while the generators are built; side_done marks their completion
  hipStream_t side = nullptr;
  hipEvent_t side_done = nullptr;
  // coupling blocks evaluated inside each product (SMASH_COUPLING_EVALUATED):
  // chunk c covers row nodes [cchunk_node[c], cchunk_node[c+1]), pairs from
  // cchunk_pair[c] and block entries from cchunk_ent[c]; Bws holds one chunk
  int coupling_mode = SMASH_COUPLING_AUTO;
  int64_t coupling_chunk = 0;
  bool coupling_eval = false;
  // evaluated form fused into the contraction (FP64 and FP32 apply): the
  // coordinates of every slot, D per slot, of the row side and the column
  // side (the same array when the column side is the row side)
  bool coupling_fused = false;
  double *xs_slot = nullptr, *ys_slot = nullptr;
  std::vector<int> cchunk_node;
  std::vector<int64_t> cchunk_pair, cchunk_ent;
  void *Bws = nullptr;
  int64_t bws_entries = 0;
  int64_t total_swaps = 0;
  // stage temporaries, released once the build has synchronised its stream
  std::vector<DeviceArena> spent;
  AllocHooks hooks;  // caller's allocator (alloc == null: the library's pool)
  double build_ms = 0;
  // product workspaces
  // captured products (options.graphs): one executable graph per argument set
  int use_graphs = 1;
  std::vector<GraphEntry> graphs;
  hipStream_t cap_stream = nullptr;
  int64_t graph_captures = 0, graph_replays = 0;
  int ws_nrhs = 0;
  void *qbuf = nullptr, *zbuf = nullptr;
  // recorded at the end of every smash_matvec product (created with the
  // handle): the next product waits for it when it runs on another stream
  // (products share the workspace), and the workspace is released only
  // after it
  hipEvent_t prod_done = nullptr;
  hipStream_t prod_stream = nullptr;
  DeviceArena ws_mem;
  MemAcct acct;              // the construction's arenas
  int64_t build_peak = 0;    // acct.peak when the construction ended
  // phase timing (options.timing)
  bool timing = false;
  struct TimedEvent {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<TimedEvent> tev;
  double phase_ms[16] = {0};
  int64_t phase_calls[16] = {0};
};

// Records a HIP event pair around the launches issued during its lifetime
// on stream s (only when the handle's timing option is on).
// Hands a stage's temporaries to the handle: work queued on the build
// stream may still read them, so they are released (to the chunk cache)
// only after the build's final stream synchronisation.
inline void defer_release(Handle &h, DeviceArena &a) {
  h.spent.push_back(a);
  a.blocks.clear();
  a.cur = nullptr;
  a.left = 0;
  a.bytes = 0;
}

struct PhaseTimer {
  Handle &h;
  int ph;
  hipStream_t s;
  hipEvent_t a = nullptr;
  PhaseTimer(Handle &h_, int ph_, hipStream_t s_) : h(h_), ph(ph_), s(s_) {
    if (h.timing && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, s);
  }
  ~PhaseTimer() {
    if (!a) return;
    hipEvent_t b;
    if (hipEventCreate(&b) == hipSuccess) {
      (void)hipEventRecord(b, s);
      h.tev.push_back({ph, a, b});
    } else {
      (void)hipEventDestroy(a);
    }
  }
};
void resolve_timers(Handle &h);

// ---------------------------------------------------------------- stages
void build_tree(Handle &h, const double *x, const double *y);
void build_pairs(Handle &h);
void build_generators(Handle &h);
// Near-field blocks: sizes and offsets (h.nboff, nLm + 1 entries), then,
// given their total, the allocation and the evaluation on h.side.
void near_offsets(Handle &h);
void near_launch(Handle &h, int64_t n_entries);
void build_blocks(Handle &h);
// Sizes and offsets of the coupling blocks (h.boff, nL + 1 entries) from the
// final ranks of both sides; the total is read with the next host read.
void coupling_offsets(Handle &h, DeviceArena &tmp);       // coupling blocks; then waits for the near ones
// coupling blocks of pairs [p0, p1) written at base + boff[p] (apply
// precision, the stored layout) on stream s
void eval_coupling_range(Handle &h, int64_t p0, int64_t p1, void *base, hipStream_t s);
void run_matvec(Handle &h, const void *X, int64_t ldx, int nrhs, void *Y, int64_t ldy,
                hipStream_t s);
// the same product with its vectors in the library's per-device array of
// SMASH_NOALLOC_SCRATCH_BYTES (no allocation, eager launches)
void run_matvec_noalloc(Handle &h, const void *X, int64_t ldx, int nrhs, void *Y, int64_t ldy,
                        hipStream_t s);
// Y = sum_l w_l o (A-hat (v_l o X)) for generators w (nx x p) and v (ny x p)
// of a Cauchy-like matrix (eqs. (6.1)-(6.2)), on stream s
void run_cauchy_like(Handle &h, const void *X, int64_t ldx, int nrhs, const double *w,
                     const double *v, int p, void *Y, int64_t ldy, hipStream_t s);
// destroys captured products (waits for each one's last launch)
void drop_graphs(Handle &h);

}  // namespace smash
