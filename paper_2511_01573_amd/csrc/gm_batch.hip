// gm_batch.hip -- batched mode: many independent integrals advanced in lock
// step through one device-resident region store (the Sec. 3 loop applied to
// every item at once).
//
// Store.  SoA centres/half-widths padded to the largest item dimension, a
// level and an item id per region.  Items are ordered by (d, family) so each
// (d, family) group owns a contiguous range of regions; each item owns a
// contiguous segment inside it, laid out exactly as its own independent run
// would lay it out (children "-" then children "+", stable order).
//
// Every segment is cut into chunks of kChunk regions (a chunk never spans
// two items), so a large item is reduced and classified by many workgroups
// instead of one wavefront.
//
// One iteration (a fixed launch sequence, replayed from a hipGraph):
//   rule      one launch per (d, family) group, the group range read on the
//             device (tile shape per group from the tuning table; the
//             degree-9 and Gauss-Kronrod rules use their own mappings)
//   reduce    one workgroup per chunk: double-double sums of Q and err
//   finalize  one wavefront per item: I, E over its chunks, T, stopping rule
//   classify  one workgroup per chunk: retire test, in-chunk ballot ranks,
//             kept count and retired sums
//   scan      one wavefront per item: chunk offsets of the kept regions,
//             retired sums, precision-limit stop
//   commit    one workgroup: shared-capacity check, commit of retired sums,
//             new segment offsets and chunk bases (scans over items)
//   scatter   halve every kept region into the other buffer
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/gm.h"
#include "gm_common.hpp"
#include "gm_internal.hpp"

namespace gm {

constexpr int kChunk = 1024;              // regions per chunk = threads per chunk workgroup
constexpr int kChunkGrid = 2048;          // grid-stride workgroups of the chunk kernels
constexpr int kMaxBatchItems = 65536;     // item slots the workspace is sized for

struct ItemState {
  int64_t off;     // segment start in the current buffer
  int64_t n;       // regions in the segment
  int64_t nk;      // kept regions this iteration
  int64_t iter;
  int32_t status;
  int32_t done;
  int32_t d;
  int32_t pad;
  int64_t regions;  // regions evaluated for this item
  int64_t off_prev;    // segment start in the buffer being split (scatter)
  int64_t cbase_prev;  // first chunk of that segment
  double I, E, T;
  double rel_tol, abs_tol;
  double ifin_hi, ifin_lo, efin_hi, efin_lo;
  double pq_hi, pq_lo, pe_hi, pe_lo;  // retired sums pending the capacity check
};

struct BatchStatus {
  int64_t n_total;    // regions in the current buffer
  int64_t n_chunks;   // chunks in the current buffer
  int64_t n_prev;     // regions in the buffer being split
  int64_t n_running;  // items still iterating
  int64_t iter;
  int64_t cap;
  int64_t max_iters;
  int64_t regions;    // regions evaluated so far
  int32_t buf;
  int32_t pad;
};

struct BatchArgs {
  BatchStatus* bst;
  ItemState* items;
  int nitems;
  int ngroups;
  const int32_t* group_first;  // first item of each group
  const int32_t* group_last;   // last item (inclusive)
  int64_t* group_range;        // [g][2] region range of each group
  double* C[2];
  double* H[2];
  uint16_t* L[2];
  uint32_t* IT[2];
  const double* Q;
  const double* ERR;
  const uint8_t* AXIS;
  int32_t* RANK;  // keep rank inside the chunk, -1 = retired
  int64_t* ICB;   // first chunk of each item's segment
  struct ChunkSums* CS;
  int64_t cap;
  int dmax;
};

// Per-chunk partial results (written by reduce / classify / scan).
struct ChunkSums {
  double q_hi, q_lo, e_hi, e_lo;  // sums of Q and err
  double rq_hi, rq_lo, re_hi, re_lo;  // sums over retired regions
  int64_t koff;  // offset of this chunk's first kept region inside the item
  int32_t kept;
  int32_t nonfinite;
};

// Item owning chunk c: the last item whose first chunk is <= c (items with no
// chunks share their successor's base, so the owner is always the last one).
__device__ __forceinline__ int chunk_item(const BatchArgs& A, int64_t c) {
  int lo = 0, hi = A.nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (A.ICB[mid] <= c) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Double-double and integer sums over a workgroup of kChunk threads; the
// result is valid in thread 0.
__device__ __forceinline__ void block_sum_chunk(dd& a, dd& b, int& k, dd* sa, dd* sb, int* sk) {
  a = wave_sum_dd(a);
  b = wave_sum_dd(b);
  k = (int)wave_sum_i64(k);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sa[w] = a;
    sb[w] = b;
    sk[w] = k;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < kChunk / 64; ++v) {
      a = dd_sum(a, sa[v]);
      b = dd_sum(b, sb[v]);
      k += sk[v];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
__global__ void batch_init_kernel(BatchArgs A, const int64_t* item_off0, const int32_t* item_m,
                                  const double* item_lo, const double* item_half, int64_t n0) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n0; r += stride) {
    if (!GM_INB(r, A.cap)) continue;
    // item of region r: last item with item_off0[i] <= r
    int lo = 0, hi = A.nitems - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (item_off0[mid] <= r) lo = mid;
      else hi = mid - 1;
    }
    const int it = lo;
    const int64_t t = r - item_off0[it];
    const int d = A.items[it].d;
    const int m = item_m[it];
    const int64_t mask = ((int64_t)1 << m) - 1;
    for (int j = 0; j < d; ++j) {
      const int64_t kj = (t >> (m * j)) & mask;
      const double hj = ldexp(item_half[it * kMaxDim + j], -m);
      A.H[0][j * A.cap + r] = hj;
      A.C[0][j * A.cap + r] = fma((double)(2 * kj + 1), hj, item_lo[it * kMaxDim + j]);
    }
    A.L[0][r] = (uint16_t)(m * d);
    A.IT[0][r] = (uint32_t)it;
  }
}

// Sums of Q and err over each chunk.
__global__ __launch_bounds__(kChunk) void batch_reduce_kernel(BatchArgs A) {
  if (A.bst->n_running == 0) return;
  __shared__ dd sa[kChunk / 64], sb[kChunk / 64];
  __shared__ int sk[kChunk / 64];
  const int64_t nc = A.bst->n_chunks;
  for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const int it = chunk_item(A, c);
    const ItemState& S = A.items[it];
    const int64_t k0 = S.off + (c - A.ICB[it]) * kChunk;
    const int64_t k1 = min(S.off + S.n, k0 + kChunk);
    const int64_t r = k0 + threadIdx.x;
    dd q = {0.0, 0.0}, e = {0.0, 0.0};
    int nf = 0;
    if (r < k1 && GM_INB(r, A.cap)) {
      q.hi = A.Q[r];
      e.hi = A.ERR[r];
      nf = (A.AXIS[r] & kNonfiniteBit) ? 1 : 0;
    }
    block_sum_chunk(q, e, nf, sa, sb, sk);
    if (threadIdx.x == 0) {
      ChunkSums& C = A.CS[c];
      C.q_hi = q.hi;
      C.q_lo = q.lo;
      C.e_hi = e.hi;
      C.e_lo = e.lo;
      C.nonfinite = nf;
    }
  }
}

// One wavefront per item: I and E over its chunks, T, the stopping rule.
__global__ __launch_bounds__(256) void batch_finalize_kernel(BatchArgs A) {
  const int lane = threadIdx.x & 63;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nw = (gridDim.x * blockDim.x) >> 6;
  if (A.bst->n_running == 0) return;
  const int64_t max_iters = A.bst->max_iters;
  for (int it = wid; it < A.nitems; it += nw) {
    ItemState& S = A.items[it];
    if (S.done) continue;
    const int64_t cb = A.ICB[it];
    const int64_t nch = (S.n + kChunk - 1) / kChunk;
    dd q = {0.0, 0.0}, e = {0.0, 0.0};
    int nonfin = 0;
    for (int64_t k = lane; k < nch; k += 64) {
      const ChunkSums& C = A.CS[cb + k];
      q = dd_sum(q, dd{C.q_hi, C.q_lo});
      e = dd_sum(e, dd{C.e_hi, C.e_lo});
      nonfin |= C.nonfinite;
    }
    q = wave_sum_dd(q);
    e = wave_sum_dd(e);
    nonfin = __any(nonfin);
    q = dd_sum(q, dd{S.ifin_hi, S.ifin_lo});
    e = dd_sum(e, dd{S.efin_hi, S.efin_lo});
    const double I = dd_val(q), E = dd_val(e);
    const int64_t iter = S.iter + 1;
    int status = -1;
    double T = 0.0;
    if (nonfin) {
      status = GM_NONFINITE;
    } else {
      T = fmax(S.abs_tol, S.rel_tol * fabs(I));
      if (E <= T) status = GM_OK;
      else if (iter >= max_iters) status = GM_MAX_ITERS;
    }
    if (lane == 0) {
      S.regions += S.n;
      S.iter = iter;
      S.I = nonfin ? NAN : I;
      S.E = nonfin ? NAN : E;
      S.T = T;
      S.nk = 0;
      if (status >= 0) {
        S.status = status;
        S.done = 1;
      }
    }
  }
}

// Classifier over each chunk of the running items: retire test, stable
// in-chunk ranks of the kept regions, kept count and retired sums.
__global__ __launch_bounds__(kChunk) void batch_classify_kernel(BatchArgs A) {
  if (A.bst->n_running == 0) return;
  __shared__ dd sa[kChunk / 64], sb[kChunk / 64];
  __shared__ int sk[kChunk / 64];
  __shared__ int wkeep[kChunk / 64];
  const int buf = A.bst->buf;
  const uint16_t* __restrict__ Lb = A.L[buf];
  const int64_t nc = A.bst->n_chunks;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const int it = chunk_item(A, c);
    const ItemState& S = A.items[it];
    if (S.done) continue;  // the same item for the whole workgroup
    const int64_t k0 = S.off + (c - A.ICB[it]) * kChunk;
    const int64_t k1 = min(S.off + S.n, k0 + kChunk);
    const int64_t r = k0 + threadIdx.x;
    const double T = S.T, aI = fabs(S.I);
    bool keep = false;
    dd fq = {0.0, 0.0}, fe = {0.0, 0.0};
    if (r < k1 && GM_INB(r, A.cap)) {
      const double err = A.ERR[r];
      const bool fin = (err <= ldexp(T, -(int)Lb[r])) || (aI + err == aI) ||
                       (A.AXIS[r] & kGeoBit);
      keep = !fin;
      if (fin) {
        fq.hi = A.Q[r];
        fe.hi = err;
      }
    }
    const uint64_t mask = __ballot(keep);
    if (lane == 0) wkeep[w] = __popcll(mask);
    __syncthreads();
    int before = 0;
    for (int v = 0; v < w; ++v) before += wkeep[v];
    if (r < k1) A.RANK[r] = keep ? before + __popcll(mask & ((1ull << lane) - 1ull)) : -1;
    int kept = keep ? 1 : 0;
    block_sum_chunk(fq, fe, kept, sa, sb, sk);
    if (threadIdx.x == 0) {
      ChunkSums& C = A.CS[c];
      C.rq_hi = fq.hi;
      C.rq_lo = fq.lo;
      C.re_hi = fe.hi;
      C.re_lo = fe.lo;
      C.kept = kept;
    }
  }
}

// One wavefront per running item: offsets of its chunks' kept regions,
// kept total, retired sums; no kept region left = precision limit.
__global__ __launch_bounds__(256) void batch_scan_kernel(BatchArgs A) {
  const int lane = threadIdx.x & 63;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nw = (gridDim.x * blockDim.x) >> 6;
  if (A.bst->n_running == 0) return;
  for (int it = wid; it < A.nitems; it += nw) {
    ItemState& S = A.items[it];
    if (S.done) continue;
    const int64_t cb = A.ICB[it];
    const int64_t nch = (S.n + kChunk - 1) / kChunk;
    int64_t run = 0;
    dd fq = {0.0, 0.0}, fe = {0.0, 0.0};
    for (int64_t k0 = 0; k0 < nch; k0 += 64) {
      const int64_t k = k0 + lane;
      int64_t kept = 0;
      if (k < nch) {
        ChunkSums& C = A.CS[cb + k];
        kept = C.kept;
        fq = dd_sum(fq, dd{C.rq_hi, C.rq_lo});
        fe = dd_sum(fe, dd{C.re_hi, C.re_lo});
      }
      int64_t inc = kept;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
      }
      if (k < nch) A.CS[cb + k].koff = run + inc - kept;
      run += __shfl(inc, 63, 64);
    }
    fq = wave_sum_dd(fq);
    fe = wave_sum_dd(fe);
    if (lane == 0) {
      S.nk = run;
      S.pq_hi = fq.hi;
      S.pq_lo = fq.lo;
      S.pe_hi = fe.hi;
      S.pe_lo = fe.lo;
      if (run == 0) {
        S.status = GM_PRECISION_LIMIT;
        S.done = 1;
      }
    }
  }
}

// Shared-capacity check, commit and new offsets (one workgroup of 1024).
__global__ __launch_bounds__(1024) void batch_commit_kernel(BatchArgs A) {
  BatchStatus* B = A.bst;
  if (B->n_running == 0) return;
  const int nit = A.nitems;
  const int per = (nit + 1023) / 1024;
  const int i0 = threadIdx.x * per;
  const int i1 = min(nit, i0 + per);
  int64_t need = 0, running = 0, chunks = 0;
  for (int i = i0; i < i1; ++i)
    if (!A.items[i].done) {
      need += 2 * A.items[i].nk;
      chunks += (2 * A.items[i].nk + kChunk - 1) / kChunk;
      running += 1;
    }
  // block reductions / scans (regions and chunks)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t inc = need, cinc = chunks;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(inc, o, 64);
    const int64_t yc = __shfl_up(cinc, o, 64);
    if (lane >= o) {
      inc += y;
      cinc += yc;
    }
  }
  __shared__ int64_t wt[16], wr[16], wc[16];
  __shared__ int over;
  const int64_t rsum = wave_sum_i64(running);
  if (lane == 63) {
    wt[w] = inc;
    wc[w] = cinc;
  }
  if (lane == 0) wr[w] = rsum;
  __syncthreads();
  int64_t woff = 0, total = 0, nrun = 0, cwoff = 0, ctotal = 0;
  for (int k = 0; k < 16; ++k) {
    if (k < w) {
      woff += wt[k];
      cwoff += wc[k];
    }
    total += wt[k];
    ctotal += wc[k];
    nrun += wr[k];
  }
  if (threadIdx.x == 0) over = (total > B->cap) ? 1 : 0;
  __syncthreads();
  if (over) {
    for (int i = i0; i < i1; ++i) {
      ItemState& S = A.items[i];
      if (!S.done) {
        S.status = GM_MAX_REGIONS;
        S.done = 1;
      }
      S.n = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      B->regions += B->n_total;
      B->n_running = 0;
      B->n_total = 0;
      for (int g = 0; g < A.ngroups; ++g) {
        A.group_range[2 * g] = 0;
        A.group_range[2 * g + 1] = 0;
      }
    }
    return;
  }
  int64_t run = woff + inc - need;
  int64_t crun = cwoff + cinc - chunks;
  for (int i = i0; i < i1; ++i) {
    ItemState& S = A.items[i];
    S.off_prev = S.off;
    S.cbase_prev = A.ICB[i];
    A.ICB[i] = crun;
    if (!S.done) {
      const dd fi = dd_sum(dd{S.ifin_hi, S.ifin_lo}, dd{S.pq_hi, S.pq_lo});
      const dd fe = dd_sum(dd{S.efin_hi, S.efin_lo}, dd{S.pe_hi, S.pe_lo});
      S.ifin_hi = fi.hi;
      S.ifin_lo = fi.lo;
      S.efin_hi = fe.hi;
      S.efin_lo = fe.lo;
      S.off = run;
      S.n = 2 * S.nk;
      run += 2 * S.nk;
      crun += (2 * S.nk + kChunk - 1) / kChunk;
    } else {
      S.off = run;
      S.n = 0;
    }
  }
  __syncthreads();
  for (int g = threadIdx.x; g < A.ngroups; g += 1024) {
    const ItemState& F = A.items[A.group_first[g]];
    const ItemState& Ls = A.items[A.group_last[g]];
    A.group_range[2 * g] = F.off;
    A.group_range[2 * g + 1] = Ls.off + Ls.n;
  }
  if (threadIdx.x == 0) {
    B->regions += B->n_total;
    B->n_prev = B->n_total;
    B->n_running = nrun;
    B->n_total = total;
    B->n_chunks = ctotal;
    B->iter += 1;
    B->buf = 1 - B->buf;
  }
}

// Split the kept regions of running items into the other buffer (runs after
// commit: the new buffer is bst->buf, the old one 1 - buf).
__global__ __launch_bounds__(256) void batch_scatter_kernel(BatchArgs A) {
  const BatchStatus* B = A.bst;
  if (B->n_running == 0) return;
  const int out = B->buf, in = 1 - out;
  const int64_t n_old = B->n_prev;
  const int64_t cap = A.cap;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_old; r += stride) {
    if (!GM_INB(r, cap)) continue;
    const uint32_t it = A.IT[in][r];
    if (!GM_INB(it, A.nitems)) continue;
    const ItemState& S = A.items[it];
    if (S.done) continue;
    const int32_t p = A.RANK[r];
    if (p < 0) continue;
    const int64_t c = S.cbase_prev + (r - S.off_prev) / kChunk;
    const int64_t pk = A.CS[c].koff + p;
    const int64_t p0 = S.off + pk, p1 = S.off + S.nk + pk;
    if (!GM_INB(p0, cap) || !GM_INB(p1, cap)) continue;
    const int ax = A.AXIS[r] & kAxisMask;
    for (int j = 0; j < S.d; ++j) {
      const double cj = A.C[in][j * cap + r];
      const double hj = A.H[in][j * cap + r];
      if (j == ax) {
        const double hp = hj * 0.5;
        A.C[out][j * cap + p0] = cj - hp;
        A.C[out][j * cap + p1] = cj + hp;
        A.H[out][j * cap + p0] = hp;
        A.H[out][j * cap + p1] = hp;
      } else {
        A.C[out][j * cap + p0] = cj;
        A.C[out][j * cap + p1] = cj;
        A.H[out][j * cap + p0] = hj;
        A.H[out][j * cap + p1] = hj;
      }
    }
    const uint16_t l1 = (uint16_t)(A.L[in][r] + 1);
    A.L[out][p0] = l1;
    A.L[out][p1] = l1;
    A.IT[out][p0] = it;
    A.IT[out][p1] = it;
  }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
namespace {

struct Tile {
  int log2l;  // -1 = one lane per region
  int grid;   // rule-kernel blocks (grid-stride)
};

std::map<int, Tile>& tile_table() {
  static std::map<int, Tile> t;
  return t;
}

int tile_key(int d, int fam) { return d * 16 + fam; }

struct BatchLayout {
  size_t C[2], H[2], L[2], IT[2], Q, ERR, AXIS, RANK, CS;
  size_t items, icb, params, vol, gfirst, glast, grange, bst, off0, m, lo, half;
  size_t total;
};

BatchLayout batch_layout(int dmax, int64_t cap, int nv, int ng) {
  BatchLayout B;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  for (int b = 0; b < 2; ++b) {
    B.C[b] = take(sizeof(double) * dmax * cap);
    B.H[b] = take(sizeof(double) * dmax * cap);
    B.L[b] = take(sizeof(uint16_t) * cap);
    B.IT[b] = take(sizeof(uint32_t) * cap);
  }
  B.Q = take(sizeof(double) * cap);
  B.ERR = take(sizeof(double) * cap);
  B.AXIS = take(cap);
  B.RANK = take(sizeof(int32_t) * cap);
  B.CS = take(sizeof(ChunkSums) * (size_t)(cap / kChunk + nv + 1));
  B.items = take(sizeof(ItemState) * nv);
  B.icb = take(sizeof(int64_t) * nv);
  B.params = take(sizeof(DevParams) * nv);
  B.vol = take(sizeof(double) * nv);
  B.gfirst = take(sizeof(int32_t) * ng);
  B.glast = take(sizeof(int32_t) * ng);
  B.grange = take(sizeof(int64_t) * 2 * ng);
  B.bst = take(sizeof(BatchStatus));
  B.off0 = take(sizeof(int64_t) * nv);
  B.m = take(sizeof(int32_t) * nv);
  B.lo = take(sizeof(double) * kMaxDim * nv);
  B.half = take(sizeof(double) * kMaxDim * nv);
  B.total = off;
  return B;
}

struct BatchNode {
  void* fn;
  dim3 grid, block;
  std::vector<void*> args;
};

}  // namespace

size_t batch_layout_bytes(int dmax, int64_t cap) {
  // per-item state for up to kMaxBatchItems items and 64 groups
  return batch_layout(dmax, cap, kMaxBatchItems, 64).total;
}

int set_tile(int d, int fam, int lanes, int grid) {
  if (d < kMinDim || d > kBatchMaxDim || fam < 1 || fam > 7 || grid < 0 || grid > 65535)
    return GM_EINVAL;
  int l = -1;
  if (lanes > 1) {
    l = 0;
    while ((1 << l) < lanes) ++l;
    if ((1 << l) != lanes) return GM_EINVAL;
  }
  if (lanes != 0 && !mapping_allowed(d, l)) return GM_EINVAL;
  if (lanes == 0) {
    tile_table().erase(tile_key(d, fam));
    return GM_OK;
  }
  tile_table()[tile_key(d, fam)] = Tile{l, grid};
  return GM_OK;
}

static Tile tile_for(int d, int fam) {
  auto it = tile_table().find(tile_key(d, fam));
  if (it != tile_table().end()) return it->second;
  return Tile{-1, 2048};
}

int run_batch(int n, const int* fam, const double* params, const int* d, const double* lo,
              const double* hi, const double* rel_tol, const double* abs_tol, int64_t cap,
              double* out_est, double* out_err, int* out_status, hipStream_t s) {
  const auto t_start = std::chrono::steady_clock::now();
  const Options& opt = options();
  if (opt.prune != 0) return GM_EINVAL;  // the batch's shared capacity has its own rule
  // Per-item offsets into the packed inputs and validation.
  std::vector<int64_t> poff(n), boff(n);
  int64_t po = 0, bo = 0;
  for (int i = 0; i < n; ++i) {
    if (d[i] < kMinDim || d[i] > kMaxDim) return GM_EINVAL;  // packing is undefined
    poff[i] = po;
    boff[i] = bo;
    po += 2 * d[i];
    bo += d[i];
  }
  std::vector<int> valid;
  for (int i = 0; i < n; ++i) {
    const bool ok = d[i] <= kBatchMaxDim &&
                    validate(fam[i], params + poff[i], d[i], lo + boff[i], hi + boff[i], rel_tol[i],
                             abs_tol[i]) == GM_OK;
    if (ok) {
      valid.push_back(i);
    } else {
      out_status[i] = GM_EINVAL;
      out_est[i] = NAN;
      out_err[i] = NAN;
    }
  }
  stats_reset();
  if (valid.empty()) return GM_OK;
  // Group items by (d, family), stable.
  std::stable_sort(valid.begin(), valid.end(), [&](int a, int b) {
    return (d[a] != d[b]) ? d[a] < d[b] : fam[a] < fam[b];
  });
  const int nv = (int)valid.size();
  std::vector<int32_t> gfirst, glast, gd, gfam;
  for (int k = 0; k < nv; ++k) {
    const int i = valid[k];
    if (k == 0 || d[i] != gd.back() || fam[i] != gfam.back()) {
      gfirst.push_back(k);
      glast.push_back(k);
      gd.push_back(d[i]);
      gfam.push_back(fam[i]);
    } else {
      glast.back() = k;
    }
  }
  const int ng = (int)gd.size();
  int dmax = 0;
  for (int k = 0; k < nv; ++k) dmax = std::max(dmax, d[valid[k]]);
  // Items, initial partition.
  std::vector<ItemState> items(nv);
  std::vector<DevParams> dparams(nv);
  std::vector<double> vol(nv), ilo((size_t)nv * kMaxDim, 0.0), ihalf((size_t)nv * kMaxDim, 0.0);
  std::vector<int64_t> off0(nv);
  std::vector<int32_t> im(nv);
  int64_t n0 = 0;
  for (int k = 0; k < nv; ++k) {
    const int i = valid[k];
    const int di = d[i];
    const int m = opt.init_log2 / di;
    std::memset(&items[k], 0, sizeof(ItemState));
    items[k].off = n0;
    items[k].n = (int64_t)1 << (m * di);
    items[k].d = di;
    items[k].rel_tol = rel_tol[i];
    items[k].abs_tol = abs_tol[i];
    fill_params(fam[i], di, params + poff[i], dparams[k]);
    double v = 1.0;
    for (int j = 0; j < di; ++j) {
      v = v * (hi[boff[i] + j] - lo[boff[i] + j]);
      ilo[(size_t)k * kMaxDim + j] = lo[boff[i] + j];
      ihalf[(size_t)k * kMaxDim + j] = (hi[boff[i] + j] - lo[boff[i] + j]) * 0.5;
    }
    vol[k] = v;
    off0[k] = n0;
    im[k] = m;
    n0 += items[k].n;
  }
  if (n0 > cap) return GM_EINVAL;
  std::vector<int64_t> icb(nv);
  int64_t nchunks0 = 0;
  for (int k = 0; k < nv; ++k) {
    icb[k] = nchunks0;
    nchunks0 += (items[k].n + kChunk - 1) / kChunk;
  }
  std::vector<int64_t> grange(2 * ng);
  for (int g = 0; g < ng; ++g) {
    grange[2 * g] = items[gfirst[g]].off;
    grange[2 * g + 1] = items[glast[g]].off + items[glast[g]].n;
  }
  const BatchLayout lay = batch_layout(dmax, cap, nv, ng);
  char* base = nullptr;
  int rc = acquire_workspace(lay.total, &base);
  if (rc != GM_OK) return rc;
  BatchStatus hb;
  std::memset(&hb, 0, sizeof hb);
  hb.n_total = n0;
  hb.n_chunks = nchunks0;
  hb.n_running = nv;
  hb.cap = cap;
  hb.max_iters = opt.max_iters;
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, s);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up(lay.items, items.data(), sizeof(ItemState) * nv);
  if (e == hipSuccess) e = up(lay.icb, icb.data(), sizeof(int64_t) * nv);
  if (e == hipSuccess) e = up(lay.params, dparams.data(), sizeof(DevParams) * nv);
  if (e == hipSuccess) e = up(lay.vol, vol.data(), sizeof(double) * nv);
  if (e == hipSuccess) e = up(lay.gfirst, gfirst.data(), sizeof(int32_t) * ng);
  if (e == hipSuccess) e = up(lay.glast, glast.data(), sizeof(int32_t) * ng);
  if (e == hipSuccess) e = up(lay.grange, grange.data(), sizeof(int64_t) * 2 * ng);
  if (e == hipSuccess) e = up(lay.bst, &hb, sizeof hb);
  if (e == hipSuccess) e = up(lay.off0, off0.data(), sizeof(int64_t) * nv);
  if (e == hipSuccess) e = up(lay.m, im.data(), sizeof(int32_t) * nv);
  if (e == hipSuccess) e = up(lay.lo, ilo.data(), sizeof(double) * kMaxDim * nv);
  if (e == hipSuccess) e = up(lay.half, ihalf.data(), sizeof(double) * kMaxDim * nv);
  if (e != hipSuccess) return record_hip_error(e);

  BatchArgs A;
  std::memset(&A, 0, sizeof A);
  A.bst = (BatchStatus*)(base + lay.bst);
  A.items = (ItemState*)(base + lay.items);
  A.nitems = nv;
  A.ngroups = ng;
  A.group_first = (const int32_t*)(base + lay.gfirst);
  A.group_last = (const int32_t*)(base + lay.glast);
  A.group_range = (int64_t*)(base + lay.grange);
  for (int b = 0; b < 2; ++b) {
    A.C[b] = (double*)(base + lay.C[b]);
    A.H[b] = (double*)(base + lay.H[b]);
    A.L[b] = (uint16_t*)(base + lay.L[b]);
    A.IT[b] = (uint32_t*)(base + lay.IT[b]);
  }
  A.Q = (const double*)(base + lay.Q);
  A.ERR = (const double*)(base + lay.ERR);
  A.AXIS = (const uint8_t*)(base + lay.AXIS);
  A.RANK = (int32_t*)(base + lay.RANK);
  A.ICB = (int64_t*)(base + lay.icb);
  A.CS = (ChunkSums*)(base + lay.CS);
  A.cap = cap;
  A.dmax = dmax;
  {
    const int g = (int)std::min<int64_t>((n0 + 255) / 256, 8192);
    hipLaunchKernelGGL(batch_init_kernel, dim3(g), dim3(256), 0, s, A,
                       (const int64_t*)(base + lay.off0), (const int32_t*)(base + lay.m),
                       (const double*)(base + lay.lo), (const double*)(base + lay.half), n0);
    e = hipGetLastError();
    if (e != hipSuccess) return record_hip_error(e);
  }
  // Kernel arguments of one iteration.
  std::vector<RuleArgs> rargs(ng);
  std::vector<RuleKernelFn> rfn(ng);
  std::vector<int> rgrid(ng);
  for (int g = 0; g < ng; ++g) {
    RuleArgs& ra = rargs[g];
    std::memset(&ra, 0, sizeof ra);
    fill_consts(gd[g], ra.K);
    ra.P.d = gd[g];
    ra.P.fam = gfam[g];
    for (int b = 0; b < 2; ++b) {
      ra.C[b] = A.C[b];
      ra.H[b] = A.H[b];
      ra.L[b] = A.L[b];
      ra.IT[b] = A.IT[b];
    }
    ra.cap = cap;
    ra.Q = (double*)(base + lay.Q);
    ra.ERR = (double*)(base + lay.ERR);
    ra.AXIS = (uint8_t*)(base + lay.AXIS);
    ra.n_fixed = -1;
    ra.PARAMS = (const DevParams*)(base + lay.params);
    ra.VOL = (const double*)(base + lay.vol);
    ra.grp = A.group_range + 2 * g;
    ra.bbuf = &A.bst->buf;
    if (opt.rule != 0) {
      // degree 9 or Gauss-Kronrod: the kernel's own mapping, a fixed
      // grid-stride grid (items of d > 6 are invalid under Gauss-Kronrod)
      rfn[g] = opt.rule == 2 ? r9_kernel(gd[g], gfam[g], true) : gk_kernel(gd[g], gfam[g], true);
      rgrid[g] = 2048;
    } else {
      const Tile t = tile_for(gd[g], gfam[g]);
      rfn[g] = rule_kernel(gd[g], gfam[g], t.log2l, true);
      rgrid[g] = t.grid > 0 ? t.grid : 2048;
    }
    if (!rfn[g]) return GM_EINVAL;
  }
  const int item_grid = (nv * 64 + 255) / 256;
  const int scat_grid = 8192;
  auto launch_iteration = [&]() -> hipError_t {
    for (int g = 0; g < ng; ++g) {
      hipLaunchKernelGGL(rfn[g], dim3(rgrid[g]), dim3(kRuleBlockSize), 0, s, rargs[g]);
    }
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(kChunkGrid), dim3(kChunk), 0, s, A);
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(item_grid), dim3(256), 0, s, A);
    hipLaunchKernelGGL(batch_classify_kernel, dim3(kChunkGrid), dim3(kChunk), 0, s, A);
    hipLaunchKernelGGL(batch_scan_kernel, dim3(item_grid), dim3(256), 0, s, A);
    hipLaunchKernelGGL(batch_commit_kernel, dim3(1), dim3(1024), 0, s, A);
    hipLaunchKernelGGL(batch_scatter_kernel, dim3(scat_grid), dim3(256), 0, s, A);
    return hipGetLastError();
  };
  // Graph of K iterations (kernel nodes only; every kernel returns at once
  // when nothing is running, so replays past the end are harmless).
  const int K = opt.graph_iters > 0 ? opt.graph_iters : 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (K > 0) {
    e = hipGraphCreate(&graph, 0);
    std::vector<hipGraphNode_t> prev;
    std::vector<void*> aptr;
    BatchArgs* Ap = &A;
    for (int k = 0; k < K && e == hipSuccess; ++k) {
      std::vector<hipGraphNode_t> rules;
      for (int g = 0; g < ng && e == hipSuccess; ++g) {
        hipKernelNodeParams p;
        std::memset(&p, 0, sizeof p);
        void* args[] = {&rargs[g]};
        p.func = (void*)rfn[g];
        p.gridDim = dim3(rgrid[g]);
        p.blockDim = dim3(kRuleBlockSize);
        p.kernelParams = args;
        hipGraphNode_t node;
        e = hipGraphAddKernelNode(&node, graph, prev.data(), prev.size(), &p);
        rules.push_back(node);
      }
      auto add = [&](void* fn, dim3 gr, dim3 bl, const std::vector<hipGraphNode_t>& dep,
                     hipGraphNode_t* node) {
        hipKernelNodeParams p;
        std::memset(&p, 0, sizeof p);
        void* args[] = {(void*)Ap};
        p.func = fn;
        p.gridDim = gr;
        p.blockDim = bl;
        p.kernelParams = args;
        return hipGraphAddKernelNode(node, graph, dep.data(), dep.size(), &p);
      };
      hipGraphNode_t n_red = nullptr, n_fin = nullptr, n_cls = nullptr, n_scan = nullptr,
                     n_commit = nullptr, n_scatter = nullptr;
      if (e == hipSuccess)
        e = add((void*)batch_reduce_kernel, dim3(kChunkGrid), dim3(kChunk), rules, &n_red);
      if (e == hipSuccess)
        e = add((void*)batch_finalize_kernel, dim3(item_grid), dim3(256), {n_red}, &n_fin);
      if (e == hipSuccess)
        e = add((void*)batch_classify_kernel, dim3(kChunkGrid), dim3(kChunk), {n_fin}, &n_cls);
      if (e == hipSuccess)
        e = add((void*)batch_scan_kernel, dim3(item_grid), dim3(256), {n_cls}, &n_scan);
      if (e == hipSuccess)
        e = add((void*)batch_commit_kernel, dim3(1), dim3(1024), {n_scan}, &n_commit);
      if (e == hipSuccess)
        e = add((void*)batch_scatter_kernel, dim3(scat_grid), dim3(256), {n_commit}, &n_scatter);
      prev = {n_scatter};
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return record_hip_error(e);
    }
  }
  const bool timing = opt.timing != 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (timing) {
    (void)hipEventCreate(&ev0);
    (void)hipEventCreate(&ev1);
  }
  double rule_ms = 0.0;
  int64_t launches = 0;
  for (int guard = 0; guard < 1000000; ++guard) {
    if (K > 0) {
      e = hipGraphLaunch(exec, s);
    } else {
      if (timing) (void)hipEventRecord(ev0, s);
      e = launch_iteration();
      if (timing) (void)hipEventRecord(ev1, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, A.bst, sizeof hb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) break;
    if (timing && K == 0) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev0, ev1);
      rule_ms += ms;
      launches += 1;
    }
    if (hb.n_running == 0) break;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (e != hipSuccess) return record_hip_error(e);
  e = hipMemcpyAsync(items.data(), A.items, sizeof(ItemState) * nv, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return record_hip_error(e);
  int worst = GM_OK;
  int64_t evals = 0, regions = 0;
  for (int k = 0; k < nv; ++k) {
    const int i = valid[k];
    out_est[i] = items[k].I;
    out_err[i] = items[k].E;
    out_status[i] = items[k].status;
    worst = std::max(worst, (int)items[k].status);
    regions += items[k].regions;
    evals += items[k].regions * nodes_per_region(items[k].d);
  }
  gm_stats& st = stats_ref();
  st.iterations = hb.iter;
  st.regions_evaluated = regions;
  st.evals = evals;
  st.status = worst;
  st.rule_ms = rule_ms;  // whole-iteration device time in direct mode
  st.rule_launches = launches;
  st.total_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  return worst;
}

GM_CHECK_UNIT(batch)

}  // namespace gm

using namespace gm;

extern "C" {

int gm_integrate_batch(int n, const int* integrand_ids, const double* params, const int* d,
                       const double* lo, const double* hi, const double* rel_tol,
                       const double* abs_tol, int64_t max_regions_total, double* out_est,
                       double* out_err, int* out_status, void* stream) {
  if (n < 1 || !integrand_ids || !params || !d || !lo || !hi || !rel_tol || !abs_tol || !out_est ||
      !out_err || !out_status || max_regions_total < 1)
    return GM_EINVAL;
  std::lock_guard<std::mutex> lk(api_mutex());
  return check_bounds(run_batch(n, integrand_ids, params, d, lo, hi, rel_tol, abs_tol,
                               max_regions_total, out_est, out_err, out_status,
                               (hipStream_t)stream));
}

int gm_set_tile(int d, int integrand_id, int lanes_per_region, int grid_blocks) {
  std::lock_guard<std::mutex> lk(api_mutex());
  return set_tile(d, integrand_id, lanes_per_region, grid_blocks);
}

}  // extern "C"
