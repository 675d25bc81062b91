// gm_api.hip -- libgm host driver (the C ABI of include/gm.h) and the control
// kernels of the breadth-first adaptive loop (arXiv 2511.01573, Sec. 3):
//
//   init      initial uniform partition into SoA storage
//   rule      (gm_rule.hip) Q, err, split axis of every active region
//   reduce    I = I_fin + sum Q, E = E_fin + sum err, T, stopping rule (Sec. 4)
//   classify  retire regions whose error share is negligible (+ guards),
//             per-tile keep counts and retired partial sums
//   scan      tile offsets of the kept regions; commit the retired sums
//   scatter   halve every kept region along its axis into the other
//             ping-pong buffer, stable order (child "-" at rank p, child "+"
//             at n_keep + p); retired leaves appended in gradient mode
//
// All iteration state lives in a device Status block; kernels read the active
// count and the ping-pong index from it and return at once when a final
// status is set, so an iteration is a fixed sequence of launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gm.h"
#include "gm_common.hpp"
#include "gm_internal.hpp"

namespace gm {

// ---------------------------------------------------------------------------
// Control kernels.
// ---------------------------------------------------------------------------
constexpr int kTile = 1024;        // regions per classify/scatter tile
constexpr int kTileThreads = 256;  // 4 regions per thread per tile
constexpr int kMaxRuleGrid = 16384;
constexpr int kPruneBins = 66;  // budget factors 2^1 .. 2^64, bin 65 = beyond
constexpr int kMaxTileGrid = 8192;
// Largest active set whose bookkeeping runs as one workgroup (small_step_kernel).
constexpr int64_t kSmallStepRegions = 4 * 1024;

struct InitArgs {
  double* C;
  double* H;
  uint16_t* L;
  int64_t cap;
  int64_t n0;
  int d;
  int m;  // cells per axis = 2^m
  double lo[kMaxDim];
  double half[kMaxDim];  // (hi - lo) / 2
};

__global__ void init_kernel(InitArgs A) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t mask = ((int64_t)1 << A.m) - 1;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < A.n0; t += stride) {
    if (!GM_INB(t, A.cap)) continue;
    for (int j = 0; j < A.d; ++j) {
      const int64_t kj = (t >> (A.m * j)) & mask;
      const double hj = ldexp(A.half[j], -A.m);
      A.H[j * A.cap + t] = hj;
      A.C[j * A.cap + t] = fma((double)(2 * kj + 1), hj, A.lo[j]);
    }
    A.L[t] = (uint16_t)(A.m * A.d);
  }
}

// Thread 0 of the reduction: the waves' sums, the retired totals, the
// iteration counters and the stopping rule (Sec. 4).
__device__ __forceinline__ void reduce_commit(Status* st, dd q, dd e, const dd* sq, const dd* se,
                                              int nw) {
  for (int w = 1; w < nw; ++w) {
    q = dd_sum(q, sq[w]);
    e = dd_sum(e, se[w]);
  }
  q = dd_sum(q, dd{st->ifin_hi, st->ifin_lo});
  e = dd_sum(e, dd{st->efin_hi, st->efin_lo});
  const double I = dd_val(q), E = dd_val(e);
  const int64_t n = st->n_active;
  st->iter += 1;
  st->regions_evaluated += n;
  if (n > st->max_active) st->max_active = n;
  if (st->nonfinite) {
    st->I = NAN;
    st->E = NAN;
    st->status = GM_NONFINITE;
    st->done = 1;
    return;
  }
  const double T = fmax(st->abs_tol, st->rel_tol * fabs(I));
  st->I = I;
  st->E = E;
  st->T = T;
  if (E <= T) {
    st->status = GM_OK;
    st->done = 1;
  } else if (st->iter >= st->max_iters) {
    st->status = GM_MAX_ITERS;
    st->done = 1;
  }
}

// Global reduction of the rule kernel's block partials and the stopping rule
// (the body of reduce_kernel and of the fused small-iteration kernel).  The
// summation order is that of kReduceLanes virtual threads whatever the block
// size (a divisor of kReduceLanes, a multiple of 64): virtual thread v adds
// partials v, v + kReduceLanes, ..., the wavefronts' sums are combined in
// order, so both kernels give the same bits.
constexpr int kReduceLanes = 1024;

__device__ __forceinline__ void reduce_body(Status* st, const double* partials, int np,
                                            int64_t* hist) {
  const int nthr = blockDim.x, tid = threadIdx.x;
  for (int b = tid; b < kPruneBins; b += nthr) hist[b] = 0;
  __shared__ dd sq[kReduceLanes / 64], se[kReduceLanes / 64];
  for (int v = tid; v < kReduceLanes; v += nthr) {
    dd q = {0.0, 0.0}, e = {0.0, 0.0};
    for (int p = v; p < np; p += kReduceLanes) {
      q = dd_sum(q, dd{partials[4 * p + 0], partials[4 * p + 1]});
      e = dd_sum(e, dd{partials[4 * p + 2], partials[4 * p + 3]});
    }
    q = wave_sum_dd(q);
    e = wave_sum_dd(e);
    if ((v & 63) == 0) {
      sq[v >> 6] = q;
      se[v >> 6] = e;
    }
  }
  __syncthreads();
  if (tid == 0) reduce_commit(st, sq[0], se[0], sq, se, kReduceLanes / 64);
}

__global__ __launch_bounds__(1024) void reduce_kernel(Status* st, const double* partials, int np,
                                                      int64_t* hist) {
  if (st->done) return;
  reduce_body(st, partials, np, hist);
}

struct ClassifyArgs {
  Status* st;
  const uint16_t* L[2];
  const double* Q;
  const double* ERR;
  const uint8_t* AXIS;
  uint8_t* FLAG;  // 1 = retired
  int64_t* TK;    // kept per tile
  double* TQ;     // retired Q per tile (double-double)
  double* TE;     // retired err per tile
  int64_t* HIST;  // kept regions per smallest sufficient budget factor (pruning)
};

// Smallest k in 1..64 with err <= T 2^(k - lvl), 65 if none: the budget factor
// that would retire the region (memory-pressure pruning).
__device__ __forceinline__ int prune_level(double err, double T, int lvl) {
  for (int k = 1; k <= 64; ++k)
    if (err <= ldexp(T, k - lvl)) return k;
  return 65;
}

// Classifier (reading of Sec. 3's "discards subregions whose contribution to
// the error is negligible"): retire when err <= T * 2^-lvl (the region's
// error density is within the global budget), when |I| + err == |I|
// (round-off guard), or when halving along the axis changes nothing
// (geometry guard, flagged by the rule kernel in bit 7 of the axis byte).
// With memory-pressure pruning on, the first pass also histograms the kept
// regions by the budget factor that would retire them; when the kept set
// overflows the store the scan kernel picks the smallest sufficient factor
// 2^k and the second pass (SECOND) classifies again with err <= T 2^(k - lvl)
// added to the retire test.
// The tiles tile0, tile0 + tstride, ... of the active set (the body of
// classify_kernel, and of the fused small-iteration kernel with one block);
// blocks of kTileThreads threads.
template <bool SECOND>
__device__ __forceinline__ void classify_tiles(const ClassifyArgs& A, int64_t tile0,
                                               int64_t tstride) {
  const Status* st = A.st;
  const int64_t n = st->n_active;
  const double T = st->T;
  const double aI = fabs(st->I);
  const int prune_k = SECOND ? st->prune_k : 0;
  const bool hist_on = !SECOND && st->prune_on;
  const uint16_t* __restrict__ L = A.L[st->buf];
  const int split = st->split;
  const int64_t npar = st->n_par;
  const int64_t nt = (n + kTile - 1) / kTile;
  __shared__ int64_t sk[kTileThreads / 64];
  __shared__ dd sq[kTileThreads / 64], se[kTileThreads / 64];
  __shared__ unsigned int shist[kPruneBins];
  if (hist_on) {
    for (int b = threadIdx.x; b < kPruneBins; b += kTileThreads) shist[b] = 0;
    __syncthreads();
  }
  for (int64_t tile = tile0; tile < nt; tile += tstride) {
    int64_t keep = 0;
    dd q = {0.0, 0.0}, e = {0.0, 0.0};
    // Every row's inputs are loaded first, by every lane (index clamped into
    // the set, Q whether or not it is needed), so the tile costs one memory
    // round trip instead of two per row (the flag stores would otherwise keep
    // the next row's loads behind them).
    constexpr int kRows = kTile / kTileThreads;
    double errv[kRows], qv[kRows];
    int lvlv[kRows];
    uint8_t axv[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int64_t r = tile * kTile + k * kTileThreads + threadIdx.x;
      const int64_t rc = r < n ? r : n - 1;
      errv[k] = A.ERR[rc];
      qv[k] = A.Q[rc];
      axv[k] = A.AXIS[rc];
      lvlv[k] = L[(split && rc >= npar) ? rc - npar : rc];  // (+ split below)
    }
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int64_t r = tile * kTile + k * kTileThreads + threadIdx.x;
      if (r < n && GM_INB(r, st->cap)) {
        const double err = errv[k];
        const int lvl = lvlv[k] + (split ? 1 : 0);
        bool fin = (err <= ldexp(T, -lvl)) || (aI + err == aI) || (axv[k] & 0x80);
        if (SECOND && !fin) fin = err <= ldexp(T, prune_k - lvl);
        if (hist_on && !fin) atomicAdd(&shist[prune_level(err, T, lvl)], 1u);
        A.FLAG[r] = fin ? 1 : 0;
        if (fin) {
          dd_add(q, qv[k]);
          dd_add(e, err);
        } else {
          keep += 1;
        }
      }
    }
    keep = wave_sum_i64(keep);
    q = wave_sum_dd(q);
    e = wave_sum_dd(e);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
      sk[w] = keep;
      sq[w] = q;
      se[w] = e;
    }
    __syncthreads();
    if (threadIdx.x == 0 && GM_INB(tile, (st->cap + kTile - 1) / kTile + 1)) {
      int64_t kk = sk[0];
      dd tq = sq[0], te = se[0];
      for (int i = 1; i < kTileThreads / 64; ++i) {
        kk += sk[i];
        tq = dd_sum(tq, sq[i]);
        te = dd_sum(te, se[i]);
      }
      A.TK[tile] = kk;
      A.TQ[2 * tile] = tq.hi;
      A.TQ[2 * tile + 1] = tq.lo;
      A.TE[2 * tile] = te.hi;
      A.TE[2 * tile + 1] = te.lo;
    }
    __syncthreads();
  }
  if (hist_on) {
    for (int b = threadIdx.x; b < kPruneBins; b += kTileThreads)
      if (shist[b]) atomicAdd((unsigned long long*)&A.HIST[b], (unsigned long long)shist[b]);
  }
}

template <bool SECOND>
__global__ __launch_bounds__(kTileThreads) void classify_kernel(ClassifyArgs A) {
  if (A.st->done) return;
  if (SECOND && !A.st->reclassify) return;
  classify_tiles<SECOND>(A, blockIdx.x, gridDim.x);
}

// Exclusive scan of the per-tile keep counts (one workgroup), capacity and
// precision checks, and the commit of the retired partial sums.  When the
// kept set overflows the store and pruning is on, the first pass picks the
// budget factor and leaves the commit to the second pass (SECOND), which runs
// after the second classification.
template <bool SECOND>
__device__ void scan_commit(Status* st, int64_t total, dd tq, dd te, const int64_t* HIST);

// Exclusive scan of the tile counts by one block (the body of scan_kernel and
// of the fused small-iteration kernel; any block size up to 1024 threads, a
// multiple of 64): thread t takes `per` consecutive tiles.
template <bool SECOND>
__device__ __forceinline__ void scan_body(Status* st, const int64_t* TK, int64_t* TOFF,
                                          const double* TQ, const double* TE,
                                          const int64_t* HIST) {
  const int nthr = blockDim.x;
  const int64_t n = st->n_active;
  const int64_t nt = (n + kTile - 1) / kTile;
  const int64_t per = (nt + nthr - 1) / nthr;
  const int64_t t0 = (int64_t)threadIdx.x * per;
  int64_t t1 = t0 + per < nt ? t0 + per : nt;
  if (t1 > t0 && !GM_INB(t1 - 1, (st->cap + kTile - 1) / kTile + 1)) t1 = t0;
  int64_t sum = 0;
  dd q = {0.0, 0.0}, e = {0.0, 0.0};
  for (int64_t t = t0; t < t1; ++t) {
    sum += TK[t];
    q = dd_sum(q, dd{TQ[2 * t], TQ[2 * t + 1]});
    e = dd_sum(e, dd{TE[2 * t], TE[2 * t + 1]});
  }
  // Inclusive scan within the wavefront.
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t inc = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  __shared__ int64_t wtot[16];
  __shared__ dd sq[16], se[16];
  q = wave_sum_dd(q);
  e = wave_sum_dd(e);
  if (lane == 63) wtot[w] = inc;
  if (lane == 0) {
    sq[w] = q;
    se[w] = e;
  }
  __syncthreads();
  int64_t woff = 0, total = 0;
  for (int i = 0; i < nthr / 64; ++i) {
    if (i < w) woff += wtot[i];
    total += wtot[i];
  }
  int64_t run = woff + inc - sum;
  for (int64_t t = t0; t < t1; ++t) {
    TOFF[t] = run;
    run += TK[t];
  }
  if (threadIdx.x != 0) return;
  dd tq = sq[0], te = se[0];
  for (int i = 1; i < nthr / 64; ++i) {
    tq = dd_sum(tq, sq[i]);
    te = dd_sum(te, se[i]);
  }
  scan_commit<SECOND>(st, total, tq, te, HIST);
}

template <bool SECOND>
__global__ __launch_bounds__(1024) void scan_kernel(Status* st, const int64_t* TK, int64_t* TOFF,
                                                    const double* TQ, const double* TE,
                                                    const int64_t* HIST) {
  if (st->done) return;
  if (SECOND && !st->reclassify) return;
  scan_body<SECOND>(st, TK, TOFF, TQ, TE, HIST);
}

// Thread 0 of the scan: capacity and precision checks, the choice of the
// pruning factor, the commit of the retired sums and the new active count.
template <bool SECOND>
__device__ void scan_commit(Status* st, int64_t total, dd tq, dd te, const int64_t* HIST) {
  const int64_t n = st->n_active;
  if (SECOND) st->reclassify = 0;
  if (total == 0) {
    // a run that pruned and then ran out of regions was limited by the store
    st->status = st->pruned ? GM_MAX_REGIONS : GM_PRECISION_LIMIT;
    st->done = 1;
    return;
  }
  if (2 * total > st->cap) {
    if (!SECOND && st->prune_on) {
      int64_t above = total;
      for (int k = 1; k <= 64; ++k) {
        above -= HIST[k];
        if (2 * above <= st->cap) {
          st->prune_k = k;
          st->pruned = 1;
          st->reclassify = 1;
          return;
        }
      }
    }
    st->status = GM_MAX_REGIONS;
    st->done = 1;
    return;
  }
  const dd fi = dd_sum(dd{st->ifin_hi, st->ifin_lo}, tq);
  const dd fe = dd_sum(dd{st->efin_hi, st->efin_lo}, te);
  st->ifin_hi = fi.hi;
  st->ifin_lo = fi.lo;
  st->efin_hi = fe.hi;
  st->efin_lo = fe.lo;
  st->finished += n - total;
  st->leaf_base = st->leaf_count;
  st->leaf_count += n - total;
  st->n_prev = n;
  st->n_keep = total;
  st->split_in = st->split;
  st->n_par_in = st->n_par;
  st->n_active = 2 * total;
  st->n_par = total;
  st->split = 1;
  st->buf = 1 - st->buf;
}

struct ScatterArgs {
  Status* st;
  double* C[2];
  double* H[2];
  uint16_t* L[2];
  uint8_t* PAX[2];
  int64_t cap;
  const uint8_t* AXIS;
  const uint8_t* FLAG;
  int64_t* TOFF;
  int d;
  // gradient mode: retired leaves (SoA, capacity leaf_cap)
  double* LC;
  double* LH;
  uint16_t* LL;
  int64_t leaf_cap;
};

// Split + stable compaction (Sec. 3: filtering and splitting fused).  Ranks
// inside a tile come from wavefront ballots and an LDS prefix over the four
// wavefronts; the tile's base offset comes from the scan kernel.  Each kept
// region is written once, at its rank p, as the record its two children are
// read from in the next iteration (centre, half-widths, level and the split
// axis the rule kernel chose); retired regions go to the leaf store in
// gradient mode.  The dimension is a template parameter so every coordinate
// load of a region is issued before its stores.  scatter_tiles takes the
// visits tile0, tile0 + tstride, ... of its tile order (the body of
// scatter_kernel and of the fused small-iteration kernel).
template <int D, bool SPLIT>
__device__ __forceinline__ void scatter_tiles_t(const ScatterArgs& A, int64_t tile0,
                                                int64_t tstride) {
  const Status* st = A.st;
  const int64_t n = st->n_prev;
  const int out = st->buf, in = 1 - out;
  const int64_t leaf_base = st->leaf_base;
  const RegionSrc R{A.C[in], A.H[in], A.L[in], A.PAX[in], A.cap, st->n_par_in, st->split_in};
  double* __restrict__ Co = A.C[out];
  double* __restrict__ Ho = A.H[out];
  uint16_t* __restrict__ Lo = A.L[out];
  uint8_t* __restrict__ Po = A.PAX[out];
  const int64_t cap = A.cap;
  const int64_t nt = (n + kTile - 1) / kTile;
  // Visiting order: the children of parent q sit at q and q + n_par, in the
  // first-half tile i and about the second-half tile m + i (m = the first
  // half's tile count).  Visit v of the grid-stride loop takes the pair's two
  // tiles at v = 16 (i / 8) + i % 8 and that + 8: blocks eight apart run on one
  // XCD (workgroups go round-robin over the eight), so the parent records that
  // the first tile reads are still in that XCD's L2 for the second.  Visits
  // past either half's end do nothing.
  const bool paired = SPLIT;
  const int64_t m = paired ? (R.npar + kTile - 1) / kTile : nt;
  const int64_t nv = paired ? 16 * ((m + 7) / 8) : nt;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __shared__ int64_t wc[kTile / kTileThreads][kTileThreads / 64];
  for (int64_t v = tile0; v < nv; v += tstride) {
    int64_t tile = v;
    if (paired) {
      const int64_t u = v >> 3, i = (u >> 1) * 8 + (v & 7);
      tile = (u & 1) ? m + i : i;
      if ((u & 1) ? tile >= nt : i >= m) continue;  // uniform over the block
    }
    // The flags of the tile's rows and its offset are loaded together (one
    // memory round trip), then the counts of every (row, wavefront), one
    // barrier per tile.
    constexpr int kRows = kTile / kTileThreads;
    uint8_t fl[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int64_t r = tile * kTile + k * kTileThreads + threadIdx.x;
      fl[k] = A.FLAG[r < n ? r : n - 1];
    }
    const int64_t tile_base = GM_INB(tile, (cap + kTile - 1) / kTile + 1) ? A.TOFF[tile] : 0;
    bool keepv[kRows];
    uint64_t masks[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int64_t r = tile * kTile + k * kTileThreads + threadIdx.x;
      keepv[k] = (r < n) && (fl[k] == 0);
      masks[k] = __ballot(keepv[k]);
      if (lane == 0) wc[k][w] = __popcll(masks[k]);
    }
    __syncthreads();
    // Destination of each row's region: rank p among the kept (parent
    // record), else its slot in the leaf store (gradient mode); -1 = none.
    // (p < cap / 2 holds by the scan's capacity check; the guards keep every
    // store inside its buffer whatever the offsets hold.)
    int64_t dst[kRows];
    {
      int64_t base = tile_base;
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        const int64_t r = tile * kTile + k * kTileThreads + threadIdx.x;
        int64_t off = base, rowtot = 0;
#pragma unroll
        for (int i = 0; i < kTileThreads / 64; ++i) {
          if (i < w) off += wc[k][i];
          rowtot += wc[k][i];
        }
        const int64_t before = off + __popcll(masks[k] & ((1ull << lane) - 1ull));
        if (keepv[k]) {
          dst[k] = GM_GUARD(before, cap) ? before : -1;
        } else {
          const int64_t slot = leaf_base + (r - before);
          dst[k] = (A.LC != nullptr && r < n && GM_GUARD(slot, A.leaf_cap)) ? slot : -1;
        }
        base += rowtot;
      }
    }
    // Records of kBatch rows are loaded before any of them is stored, so a
    // wavefront has that many rows' reads in flight at once.
    constexpr int kBatch = D <= 8 ? 4 : D <= 12 ? 2 : 1;
#pragma unroll
    for (int k0 = 0; k0 < kRows; k0 += kBatch) {
      // Every lane loads (the index clamped into the set), so no loaded
      // value is merged across a branch before its use: the waits for a
      // batch's loads come only at its stores.
      double gc[kBatch][D], gh[kBatch][D];
      uint16_t gl[kBatch];
      uint8_t gp[kBatch], ga[kBatch];
      bool gplus[kBatch];
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int64_t r0 = tile * kTile + (k0 + b) * kTileThreads + threadIdx.x;
        const int64_t r = r0 < n ? r0 : n - 1;
        gplus[b] = SPLIT && r >= R.npar;
        int64_t q = gplus[b] ? r - R.npar : r;
        if (!GM_INB(q, cap)) q = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          gc[b][j] = R.C[j * cap + q];
          gh[b][j] = R.H[j * cap + q];
        }
        gl[b] = R.L[q];
        gp[b] = SPLIT ? R.PAX[q] : 0;
        ga[b] = A.AXIS[r];
      }
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int k = k0 + b;
        const int64_t p = dst[k];
        if (p < 0) continue;
        // the child: the parent's split axis halved, the centre moved
        double c[D], h[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          c[j] = gc[b][j];
          h[j] = gh[b][j];
          if (SPLIT && j == gp[b]) {
            const double hp = gh[b][j] * 0.5;
            c[j] = gplus[b] ? gc[b][j] + hp : gc[b][j] - hp;
            h[j] = hp;
          }
        }
        const int lvl = SPLIT ? gl[b] + 1 : gl[b];
        if (keepv[k]) {
#pragma unroll
          for (int j = 0; j < D; ++j) {
            Co[j * cap + p] = c[j];
            Ho[j * cap + p] = h[j];
          }
          Lo[p] = (uint16_t)lvl;
          Po[p] = ga[b] & kAxisMask;
        } else {
#pragma unroll
          for (int j = 0; j < D; ++j) {
            A.LC[j * A.leaf_cap + p] = c[j];
            A.LH[j * A.leaf_cap + p] = h[j];
          }
          A.LL[p] = (uint16_t)lvl;
        }
      }
    }
    __syncthreads();
  }
}

// (SPLIT: the input set is stored as parent records, as after every
// iteration but the first.)
template <int D>
__device__ __forceinline__ void scatter_tiles(const ScatterArgs& A, int64_t tile0,
                                              int64_t tstride) {
  if (A.st->split_in)
    scatter_tiles_t<D, true>(A, tile0, tstride);
  else
    scatter_tiles_t<D, false>(A, tile0, tstride);
}

template <int D>
__global__ __launch_bounds__(kTileThreads) void scatter_kernel(ScatterArgs A) {
  if (A.st->done) return;
  scatter_tiles<D>(A, blockIdx.x, gridDim.x);
}

// One iteration's bookkeeping for a small active set in a single workgroup:
// the reduction and stopping rule, the classification, the scan and the
// split + compaction of reduce_kernel, classify_kernel<false>, scan_kernel<false>
// and scatter_kernel, in that order and with the same results, separated by
// workgroup barriers instead of kernel boundaries (for active sets of a few
// tiles the four launches cost more than their work).  Not for memory-
// pressure pruning (its second classification pass).
template <int D>
__global__ __launch_bounds__(kTileThreads) void small_step_kernel(Status* st,
                                                                  const double* partials, int np,
                                                                  ClassifyArgs ca, ScatterArgs sa) {
  if (st->done) return;
  reduce_body(st, partials, np, ca.HIST);
  __syncthreads();
  if (st->done) return;
  classify_tiles<false>(ca, 0, 1);
  __syncthreads();
  scan_body<false>(st, ca.TK, sa.TOFF, ca.TQ, ca.TE, ca.HIST);
  __syncthreads();
  if (st->done) return;
  scatter_tiles<D>(sa, 0, 1);
}

using ScatterFn = void (*)(ScatterArgs);
using SmallStepFn = void (*)(Status*, const double*, int, ClassifyArgs, ScatterArgs);

static ScatterFn scatter_fn(int d) {
  switch (d) {
    case 2: return scatter_kernel<2>;
    case 3: return scatter_kernel<3>;
    case 4: return scatter_kernel<4>;
    case 5: return scatter_kernel<5>;
    case 6: return scatter_kernel<6>;
    case 7: return scatter_kernel<7>;
    case 8: return scatter_kernel<8>;
    case 9: return scatter_kernel<9>;
    case 10: return scatter_kernel<10>;
    case 11: return scatter_kernel<11>;
    case 12: return scatter_kernel<12>;
    case 13: return scatter_kernel<13>;
    case 14: return scatter_kernel<14>;
    case 15: return scatter_kernel<15>;
    case 16: return scatter_kernel<16>;
    default: return nullptr;
  }
}

static SmallStepFn small_step_fn(int d) {
  switch (d) {
    case 2: return small_step_kernel<2>;
    case 3: return small_step_kernel<3>;
    case 4: return small_step_kernel<4>;
    case 5: return small_step_kernel<5>;
    case 6: return small_step_kernel<6>;
    case 7: return small_step_kernel<7>;
    case 8: return small_step_kernel<8>;
    case 9: return small_step_kernel<9>;
    case 10: return small_step_kernel<10>;
    case 11: return small_step_kernel<11>;
    case 12: return small_step_kernel<12>;
    case 13: return small_step_kernel<13>;
    case 14: return small_step_kernel<14>;
    case 15: return small_step_kernel<15>;
    case 16: return small_step_kernel<16>;
    default: return nullptr;
  }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
namespace {

Options g_opt;
gm_stats g_stats;
std::string g_hip_err = "no HIP error";
std::string g_enomem_text;

// Device memory: either the caller's registered workspace or a cached
// library allocation that only grows.
void* g_ext_ptr = nullptr;
size_t g_ext_bytes = 0;
void* g_own_ptr = nullptr;
size_t g_own_bytes = 0;

// The last run, for gm_last_active.
struct LastRun {
  bool valid = false;
  int d = 0;
  int64_t n = 0, cap = 0;
  int64_t npar = 0;  // records behind a split set
  int split = 0;
  Layout lay;
  int buf = 0;
  char* base = nullptr;  // device buffers of that run
} g_last;

int hip_fail(hipError_t e) {
  g_hip_err = hipGetErrorString(e);
  (void)hipGetLastError();
  return GM_EHIP;
}

#define GM_HIP(call)                      \
  do {                                    \
    hipError_t _e = (call);               \
    if (_e != hipSuccess) return hip_fail(_e); \
  } while (0)

}  // namespace

Options& options() { return g_opt; }

std::mutex& api_mutex() {
  static std::mutex mu;
  return mu;
}

int record_hip_error(hipError_t e) { return hip_fail(e); }

GM_CHECK_UNIT(api)

#ifdef GM_CHECK
// Self-test of the check path: one index one past its bound, checked and not
// used (no memory is accessed).
__global__ void check_selftest_kernel(int64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) (void)GM_INB(n, n);
}

int check_bounds(int rc) {
  using PollFn = int (*)(CheckRec*);
#define GM_POLL_F(name)                                                               \
  {#name " f1", gm_check_poll_##name##_f1}, {#name " f2", gm_check_poll_##name##_f2}, \
  {#name " f3", gm_check_poll_##name##_f3}, {#name " f4", gm_check_poll_##name##_f4}, \
  {#name " f5", gm_check_poll_##name##_f5}, {#name " f6", gm_check_poll_##name##_f6}, \
  {#name " f7", gm_check_poll_##name##_f7}
  static const struct {
    const char* name;
    PollFn fn;
  } units[] = {{"api", gm_check_poll_api}, {"batch", gm_check_poll_batch},
               {"grad", gm_check_poll_grad}, GM_POLL_F(rule), GM_POLL_F(rule9),
               GM_POLL_F(adjoint), GM_POLL_F(gk)};
#undef GM_POLL_F
  std::string first;
  unsigned long long total = 0;
  for (const auto& u : units) {
    CheckRec r = {};
    if (u.fn(&r) != 0) return hip_fail(hipGetLastError());
    if (r.count != 0 && first.empty()) {
      char buf[256];
      std::snprintf(buf, sizeof buf, "bounds check failed in unit %s, line %d: index %lld, bound %lld",
                    u.name, r.line, r.index, r.bound);
      first = buf;
    }
    total += r.count;
  }
  if (total == 0) return rc;
  g_hip_err = first + " (" + std::to_string(total) + " violations)";
  return GM_EHIP;
}
#else
int check_bounds(int rc) { return rc; }
#endif

void stats_reset() { std::memset(&g_stats, 0, sizeof g_stats); }
gm_stats& stats_ref() { return g_stats; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout make_layout(int d, int64_t cap) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  const int64_t ntiles = (cap + kTile - 1) / kTile + 1;
  for (int b = 0; b < 2; ++b) {
    L.C[b] = take(sizeof(double) * d * cap);
    L.H[b] = take(sizeof(double) * d * cap);
    L.L[b] = take(sizeof(uint16_t) * cap);
    L.PAX[b] = take(cap);
  }
  L.Q = take(sizeof(double) * cap);
  L.ERR = take(sizeof(double) * cap);
  L.AXIS = take(cap);
  L.FLAG = take(cap);
  L.TK = take(sizeof(int64_t) * ntiles);
  L.TOFF = take(sizeof(int64_t) * ntiles);
  L.TQ = take(sizeof(double) * 2 * ntiles);
  L.TE = take(sizeof(double) * 2 * ntiles);
  L.PART = take(sizeof(double) * 4 * kMaxRuleGrid);
  L.ST = take(sizeof(Status));
  L.HIST = take(sizeof(int64_t) * kPruneBins);
  L.total = off;
  return L;
}

int acquire_workspace(size_t bytes, char** base) {
  if (g_ext_ptr) {
    if (bytes > g_ext_bytes) return GM_ENOMEM;
    *base = (char*)g_ext_ptr;
    return GM_OK;
  }
  if (bytes > g_own_bytes) {
    g_last.valid = false;  // the last run's buffers go away
    if (g_own_ptr) {
      GM_HIP(hipDeviceSynchronize());
      GM_HIP(hipFree(g_own_ptr));
      g_own_ptr = nullptr;
      g_own_bytes = 0;
    }
    hipError_t e = hipMalloc(&g_own_ptr, bytes);
    if (e != hipSuccess) {
      g_hip_err = hipGetErrorString(e);
      (void)hipGetLastError();
      g_own_ptr = nullptr;
      return GM_ENOMEM;
    }
    g_own_bytes = bytes;
  }
  *base = (char*)g_own_ptr;
  return GM_OK;
}

void fill_consts(int d, RuleConsts& K) {
  const int64_t D = d;
  K.lam2 = std::sqrt(9.0 / 70.0);
  K.lam3 = std::sqrt(9.0 / 10.0);
  K.lam4 = std::sqrt(9.0 / 10.0);
  K.lam5 = std::sqrt(9.0 / 19.0);
  K.w[0] = (double)(400 * D * D - 9120 * D + 12824) / 19683.0;
  K.w[1] = 980.0 / 6561.0;
  K.w[2] = (double)(1820 - 400 * D) / 19683.0;
  K.w[3] = 200.0 / 19683.0;
  K.w[4] = std::ldexp(6859.0 / 19683.0, -d);
  K.e[0] = (double)(-19 * (50 * D * D - 870 * D + 361)) / 19683.0;
  K.e[1] = -4655.0 / 13122.0;
  K.e[2] = (double)(95 * (20 * D - 37)) / 39366.0;
  K.e[3] = -475.0 / 19683.0;
  K.e[4] = K.w[4];
  K.r7 = 1.0 / 7.0;
  K.axis_band = 1e-10;
  // degree-9 rule: the unique solution of its even-moment equations (degree
  // <= 8), each weight one correctly rounded division of exact integers
  K.lam6 = std::sqrt(759.0 / 1190.0);
  K.w9[0] = (double)(-160 * (6325 * D * D * D - 345345 * D * D + 1801355 * D - 1902813)) /
            403363719.0;
  K.w9[1] = (double)(-490 * (2020 * D - 8711)) / 17891847.0;
  K.w9[2] = (double)(5 * (10400 * D * D - 236080 * D + 404019)) / 13817466.0;
  K.w9[3] = (double)(-1000 * (2 * D - 9)) / 531441.0;
  K.w9[4] = std::ldexp(130321.0 / 531441.0, -d);
  K.w9[5] = 20462645.0 / 484331562.0;
  K.w9[6] = 4900.0 / 177147.0;
  K.w9[7] = 1000.0 / 531441.0;
  // minus the degree-7 weights (zero on classes 6..8), exact, rounded once
  K.e9[0] = (double)(-8 * (126500 * D * D * D - 5882250 * D * D + 12665080 * D - 5205981)) /
            403363719.0;
  K.e9[1] = (double)(-490 * (2020 * D - 3257)) / 17891847.0;
  K.e9[2] = (double)(5 * (10400 * D * D - 179920 * D + 148491)) / 13817466.0;
  K.e9[3] = (double)(-400 * (5 * D - 9)) / 531441.0;
  K.e9[4] = std::ldexp(-54872.0 / 531441.0, -d);
  K.e9[5] = K.w9[5];
  K.e9[6] = K.w9[6];
  K.e9[7] = K.w9[7];
  // degree-3 rule on the centre and the +-l3 e_i nodes (exact on 1 and x^2)
  K.q3[0] = (double)(27 - 10 * D) / 27.0;
  K.q3[1] = 5.0 / 27.0;
  K.err_model = g_opt.err_model;
}

void fill_params(int fam, int d, const double* params, DevParams& P) {
  std::memset(&P, 0, sizeof P);
  P.d = d;
  P.fam = fam;
  for (int j = 0; j < d; ++j) {
    P.a[j] = params[j];
    P.u[j] = params[d + j];
    P.inv_a2[j] = 1.0 / (P.a[j] * P.a[j]);
  }
  P.c0 = 6.283185307179586476925286766559 * P.u[0];
}

int validate(int fam, const double* params, int d, const double* lo, const double* hi,
             double rel_tol, double abs_tol) {
  if (fam < 1 || fam > 7) return GM_EINVAL;
  if (d < kMinDim || d > kMaxDim) return GM_EINVAL;
  if (!params || !lo || !hi) return GM_EINVAL;
  if (!(rel_tol >= 0.0) || !(abs_tol >= 0.0) || !std::isfinite(rel_tol) || !std::isfinite(abs_tol))
    return GM_EINVAL;
  if (rel_tol == 0.0 && abs_tol == 0.0) return GM_EINVAL;
  if (g_opt.rule == 1 && d > kGkMaxDim) return GM_EINVAL;
  for (int j = 0; j < d; ++j)
    if (!std::isfinite(lo[j]) || !std::isfinite(hi[j]) || !(lo[j] < hi[j])) return GM_EINVAL;
  for (int j = 0; j < 2 * d; ++j)
    if (!std::isfinite(params[j])) return GM_EINVAL;
  return GM_OK;
}

int init_cells_log2(int d) { return g_opt.init_log2 / d; }

RuleKernelFn rule_kernel(int d, int fam, int log2l, bool batch) {
  switch (fam) {
    case 1: return rule_kernel_f1(d, log2l, batch);
    case 2: return rule_kernel_f2(d, log2l, batch);
    case 3: return rule_kernel_f3(d, log2l, batch);
    case 4: return rule_kernel_f4(d, log2l, batch);
    case 5: return rule_kernel_f5(d, log2l, batch);
    case 6: return rule_kernel_f6(d, log2l, batch);
    case 7: return rule_kernel_f7(d, log2l, batch);
    default: return nullptr;
  }
}

RuleKernelFn gk_kernel(int d, int fam, bool batch) {
  switch (fam) {
    case 1: return gk_kernel_f1(d, batch);
    case 2: return gk_kernel_f2(d, batch);
    case 3: return gk_kernel_f3(d, batch);
    case 4: return gk_kernel_f4(d, batch);
    case 5: return gk_kernel_f5(d, batch);
    case 6: return gk_kernel_f6(d, batch);
    case 7: return gk_kernel_f7(d, batch);
    default: return nullptr;
  }
}

RuleKernelFn r9_kernel(int d, int fam, bool batch, bool wide) {
  switch (fam) {
    case 1: return rule9_kernel_f1(d, batch, wide);
    case 2: return rule9_kernel_f2(d, batch, wide);
    case 3: return rule9_kernel_f3(d, batch, wide);
    case 4: return rule9_kernel_f4(d, batch, wide);
    case 5: return rule9_kernel_f5(d, batch, wide);
    case 6: return rule9_kernel_f6(d, batch, wide);
    case 7: return rule9_kernel_f7(d, batch, wide);
    default: return nullptr;
  }
}

// Mapping codes: the Gauss-Kronrod kernel (gk_threads(d) per region), and the
// degree-9 kernel with 2^(code - kMapR9) lanes per region.
constexpr int kMapGk = 100;
constexpr int kMapR9 = 200;

int lanes_of_mapping(int map, int d) {
  return map == kMapGk ? gk_threads(d) : map >= kMapR9 ? (1 << (map - kMapR9)) : map < 0 ? 1 : (1 << map);
}

int64_t nodes_per_region(int d) {
  if (g_opt.rule == 1) {
    int64_t n = 1;
    for (int j = 0; j < d; ++j) n *= 15;
    return n;
  }
  if (g_opt.rule == 2) {
    const int64_t D = d;
    return 1 + 6 * D + 6 * D * (D - 1) + 4 * D * (D - 1) * (D - 2) / 3 + ((int64_t)1 << d);
  }
  return gm_num_nodes(d);
}

hipError_t launch_rule(int d, int fam, int log2l, const RuleArgs& a, int grid, hipStream_t s) {
  RuleKernelFn fn = log2l == kMapGk    ? gk_kernel(d, fam, false)
                    : log2l >= kMapR9 ? r9_kernel(d, fam, false, log2l - kMapR9 != rule9_log2l(d))
                                      : rule_kernel(d, fam, log2l, false);
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kRuleBlockSize), 0, s, a);
  return hipGetLastError();
}

bool mapping_allowed(int d, int log2l) {
  if (log2l < 0) return d <= kTprMaxDim;
  if (log2l == 2) return d >= 6;
  if (log2l == 4) return d >= 8;
  if (log2l == 6) return d >= 10;
  return false;
}

// Lanes the rule kernel should occupy: 256 CUs x 4 SIMDs x 2 wavefronts x 64.
constexpr int64_t kTargetLanes = 131072;

int choose_mapping(int d, int64_t n) {
  if (g_opt.rule == 1) return kMapGk;
  if (g_opt.rule == 2) {
    // the wide mapping while the default one would leave the GPU mostly idle
    const bool wide = (n << rule9_log2l(d)) < kTargetLanes;
    return kMapR9 + (wide ? rule9_log2l_wide(d) : rule9_log2l(d));
  }
  const int forced = g_opt.lanes_per_region;
  if (forced > 0) {
    int l = -1;
    if (forced > 1) {
      l = 0;
      while ((1 << l) < forced) ++l;
    }
    if (mapping_allowed(d, l)) return l;
  }
  const int cands[4] = {-1, 2, 4, 6};
  int best = -2;
  for (int k = 0; k < 4; ++k) {
    const int l = cands[k];
    if (!mapping_allowed(d, l)) continue;
    best = l;
    const int64_t lanes = (l < 0) ? n : (n << l);
    if (lanes >= kTargetLanes) break;
  }
  return best;
}

int rule_grid(int log2l, int64_t n, int d) {
  const int64_t per_block = log2l == kMapGk    ? kRuleBlockSize / gk_threads(d)
                            : log2l >= kMapR9 ? (kRuleBlockSize >> (log2l - kMapR9))
                            : (log2l < 0)   ? kRuleBlockSize
                                            : (kRuleBlockSize >> log2l);
  const int64_t g = (n + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, kMaxRuleGrid));
}

static int tile_grid_for(int64_t n) {
  int64_t g = (n + kTile - 1) / kTile;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, kMaxTileGrid));
}

// Grid of the split + compaction: its paired visiting order (scatter_tiles)
// has up to 16 * ceil(ceil(n / 2 / kTile) / 8) visits for n regions.
static int scatter_grid_for(int64_t n) {
  const int64_t m = (n / 2 + kTile - 1) / kTile + 1;
  const int64_t g = std::max<int64_t>((n + kTile - 1) / kTile, 16 * ((m + 7) / 8));
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, kMaxTileGrid));
}

// Leaf store of the gradient mode (SoA, grows on demand).
struct LeafStore {
  double* C = nullptr;
  double* H = nullptr;
  uint16_t* L = nullptr;
  int64_t cap = 0;
  int d = 0;
  void release() {
    if (C) (void)hipFree(C);
    if (H) (void)hipFree(H);
    if (L) (void)hipFree(L);
    C = H = nullptr;
    L = nullptr;
    cap = 0;
  }
};

static LeafStore g_leaves;

LeafView leaf_view() { return LeafView{g_leaves.C, g_leaves.H, g_leaves.L, g_leaves.cap}; }

static int leaf_reserve(int d, int64_t need, int64_t have, hipStream_t s) {
  if (need <= g_leaves.cap && g_leaves.d == d) return GM_OK;
  // A store of another dimension holds nothing to keep: free it first and
  // size the new one from this run's need alone (doubling its capacity would
  // compound over calls that alternate dimensions).
  if (g_leaves.d != d) {
    GM_HIP(hipStreamSynchronize(s));
    g_leaves.release();
    g_leaves.d = d;
    have = 0;
  }
  int64_t nc = std::max<int64_t>(need, std::max<int64_t>(1 << 16, 2 * g_leaves.cap));
  double *C = nullptr, *H = nullptr;
  uint16_t* L = nullptr;
  if (hipMalloc(&C, sizeof(double) * d * nc) != hipSuccess ||
      hipMalloc(&H, sizeof(double) * d * nc) != hipSuccess ||
      hipMalloc(&L, sizeof(uint16_t) * nc) != hipSuccess) {
    (void)hipGetLastError();
    if (C) (void)hipFree(C);
    if (H) (void)hipFree(H);
    if (L) (void)hipFree(L);
    return GM_ENOMEM;
  }
  if (have > 0) {
    for (int j = 0; j < d; ++j) {
      GM_HIP(hipMemcpyAsync(C + j * nc, g_leaves.C + j * g_leaves.cap, sizeof(double) * have,
                            hipMemcpyDeviceToDevice, s));
      GM_HIP(hipMemcpyAsync(H + j * nc, g_leaves.H + j * g_leaves.cap, sizeof(double) * have,
                            hipMemcpyDeviceToDevice, s));
    }
    GM_HIP(hipMemcpyAsync(L, g_leaves.L, sizeof(uint16_t) * have, hipMemcpyDeviceToDevice, s));
    GM_HIP(hipStreamSynchronize(s));
  }
  g_leaves.release();
  g_leaves.C = C;
  g_leaves.H = H;
  g_leaves.L = L;
  g_leaves.cap = nc;
  g_leaves.d = d;
  return GM_OK;
}

// Pinned host copy of the status block: the host's status reads and the
// initial write are direct DMA transfers instead of staged pageable copies.
// create = false returns the copy only if an earlier call made it.
static Status* pinned_status(bool create = true) {
  static Status* p = nullptr;
  if (!p && create &&
      hipHostMalloc((void**)&p, sizeof(Status), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  return p;
}

// Fixed device scratch of gm_integrate_noalloc (callers that cannot allocate):
// a file-scope array each device holds until the process ends.  In host code
// `scratch` names a host-side stand-in, never the device address: the address
// is looked up once per device with hipGetSymbolAddress (that device current)
// and only that pointer is handed to kernels and copies.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
constexpr int kMaxDevices = 64;
static char* g_scratch_dev[kMaxDevices] = {};

static int noalloc_scratch(char** out) {
  int dev = 0;
  GM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    g_hip_err = "device index beyond the no-allocation scratch table";
    return GM_EHIP;
  }
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    GM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255u) != 0) {
      g_hip_err = "no-allocation scratch: unexpected device address";
      return GM_EHIP;
    }
    g_scratch_dev[dev] = (char*)p;
  }
  *out = g_scratch_dev[dev];
  return GM_OK;
}

// One adaptive run on the device (gm_integrate and the forward pass of
// gm_integrate_grad).  On return the status block holds the final state.
int run_adaptive(int fam, const double* params, int d, const double* lo, const double* hi,
                 double rel_tol, double abs_tol, int64_t max_regions, hipStream_t s,
                 bool keep_leaves, RunResult* out, char* fixed_base) {
  const auto t_start = std::chrono::steady_clock::now();
  std::memset(&g_stats, 0, sizeof g_stats);
  const int m = init_cells_log2(d);
  const int64_t n0 = (int64_t)1 << (m * d);
  if (max_regions < n0) return GM_EINVAL;
  const int64_t cap = max_regions;
  const Layout lay = make_layout(d, cap);
  g_last.valid = false;  // (before the workspace may move)
  char* base = fixed_base;
  int rc = GM_OK;
  if (!base) {
    rc = acquire_workspace(lay.total, &base);
    if (rc != GM_OK) return rc;
  }

  RuleArgs ra;
  std::memset(&ra, 0, sizeof ra);
  fill_params(fam, d, params, ra.P);
  fill_consts(d, ra.K);
  for (int b = 0; b < 2; ++b) {
    ra.C[b] = (const double*)(base + lay.C[b]);
    ra.H[b] = (const double*)(base + lay.H[b]);
    ra.L[b] = (const uint16_t*)(base + lay.L[b]);
    ra.PAX[b] = (const uint8_t*)(base + lay.PAX[b]);
  }
  ra.cap = cap;
  ra.Q = (double*)(base + lay.Q);
  ra.ERR = (double*)(base + lay.ERR);
  ra.AXIS = (uint8_t*)(base + lay.AXIS);
  ra.partials = (double*)(base + lay.PART);
  Status* st = (Status*)(base + lay.ST);
  ra.st = st;
  double vol = 1.0;
  for (int j = 0; j < d; ++j) vol = vol * (hi[j] - lo[j]);
  ra.vol_omega = vol;
  ra.n_fixed = -1;

  InitArgs ia;
  std::memset(&ia, 0, sizeof ia);
  ia.C = (double*)ra.C[0];
  ia.H = (double*)ra.H[0];
  ia.L = (uint16_t*)ra.L[0];
  ia.cap = cap;
  ia.n0 = n0;
  ia.d = d;
  ia.m = m;
  for (int j = 0; j < d; ++j) {
    ia.lo[j] = lo[j];
    ia.half[j] = (hi[j] - lo[j]) * 0.5;
  }

  ClassifyArgs ca;
  ca.st = st;
  ca.L[0] = ra.L[0];
  ca.L[1] = ra.L[1];
  ca.Q = ra.Q;
  ca.ERR = ra.ERR;
  ca.AXIS = ra.AXIS;
  ca.FLAG = (uint8_t*)(base + lay.FLAG);
  ca.TK = (int64_t*)(base + lay.TK);
  ca.TQ = (double*)(base + lay.TQ);
  ca.TE = (double*)(base + lay.TE);
  ca.HIST = (int64_t*)(base + lay.HIST);

  ScatterArgs sa;
  std::memset(&sa, 0, sizeof sa);
  sa.st = st;
  for (int b = 0; b < 2; ++b) {
    sa.C[b] = (double*)ra.C[b];
    sa.H[b] = (double*)ra.H[b];
    sa.L[b] = (uint16_t*)ra.L[b];
    sa.PAX[b] = (uint8_t*)ra.PAX[b];
  }
  sa.cap = cap;
  sa.AXIS = ra.AXIS;
  sa.FLAG = ca.FLAG;
  sa.TOFF = (int64_t*)(base + lay.TOFF);
  sa.d = d;

  Status hst;
  std::memset(&hst, 0, sizeof hst);
  hst.n_active = n0;
  hst.cap = cap;
  hst.max_iters = g_opt.max_iters;
  hst.rel_tol = rel_tol;
  hst.abs_tol = abs_tol;
  hst.prune_on = g_opt.prune;
  Status* const pin = pinned_status(fixed_base == nullptr);
  if (pin) {
    *pin = hst;
    GM_HIP(hipMemcpyAsync(st, pin, sizeof hst, hipMemcpyHostToDevice, s));
  } else {
    GM_HIP(hipMemcpyAsync(st, &hst, sizeof hst, hipMemcpyHostToDevice, s));
  }
  {
    int g = (int)std::min<int64_t>((n0 + 255) / 256, 4096);
    hipLaunchKernelGGL(init_kernel, dim3(g), dim3(256), 0, s, ia);
    GM_HIP(hipGetLastError());
  }

  // Iterations launched back to back before the host reads the status
  // block (6 while the active set is below 2^16 regions, 3 below 2^20, 2
  // above): kernels take the active count from the device and return at once
  // after a final status, so launches past the end cost only their launch.
  // Grids are sized for the largest count the iteration can have (n doubles
  // at most per iteration).  Gradient mode checks every iteration (the leaf
  // store grows on the host's side).
  constexpr int kMaxAhead = 8;
  hipEvent_t ev[kMaxAhead][5] = {};
  // (events are created per run: not on the no-allocation path)
  const bool timing = g_opt.timing != 0 && !fixed_base;  // rule kernel only
  const bool phases = timing && g_opt.timing >= 2;       // every phase
  if (timing)
    for (auto& row : ev)
      for (auto& e : row) GM_HIP(hipEventCreate(&e));

  int64_t n = n0;
  int64_t leaves_have = 0;
  int64_t iter_done = 0;
  for (;;) {
    int K = 1;
    if (!keep_leaves)
      K = g_opt.graph_iters > 0 ? std::min(g_opt.graph_iters, kMaxAhead) : (n < (1 << 16) ? 6 : n < (1 << 20) ? 3 : 2);
    if (keep_leaves) {
      // Room for every region of this iteration to retire.
      rc = leaf_reserve(d, leaves_have + n, leaves_have, s);
      if (rc != GM_OK) return rc;
      sa.LC = g_leaves.C;
      sa.LH = g_leaves.H;
      sa.LL = g_leaves.L;
      sa.leaf_cap = g_leaves.cap;
    }
    int64_t nb = n;
    for (int k = 0; k < K; ++k) {
      const int map = choose_mapping(d, nb);
      const int rg = rule_grid(map, nb, d);
      const int tg = tile_grid_for(nb);
      g_stats.lanes_per_region = lanes_of_mapping(map, d);
      if (timing) GM_HIP(hipEventRecord(ev[k][0], s));
      GM_HIP(launch_rule(d, fam, map, ra, rg, s));
      if (timing) GM_HIP(hipEventRecord(ev[k][1], s));
      if (!g_opt.prune && !phases && nb <= kSmallStepRegions) {
        hipLaunchKernelGGL(small_step_fn(d), dim3(1), dim3(kTileThreads), 0, s, st, ra.partials,
                           rg, ca, sa);
        GM_HIP(hipGetLastError());
        nb = std::min<int64_t>(cap, 2 * nb);
        continue;
      }
      hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, s, st, ra.partials, rg, ca.HIST);
      GM_HIP(hipGetLastError());
      if (phases) GM_HIP(hipEventRecord(ev[k][2], s));
      hipLaunchKernelGGL(classify_kernel<false>, dim3(tg), dim3(kTileThreads), 0, s, ca);
      GM_HIP(hipGetLastError());
      if (phases) GM_HIP(hipEventRecord(ev[k][3], s));
      hipLaunchKernelGGL(scan_kernel<false>, dim3(1), dim3(1024), 0, s, st, ca.TK, sa.TOFF, ca.TQ,
                         ca.TE, ca.HIST);
      GM_HIP(hipGetLastError());
      if (g_opt.prune) {
        hipLaunchKernelGGL(classify_kernel<true>, dim3(tg), dim3(kTileThreads), 0, s, ca);
        GM_HIP(hipGetLastError());
        hipLaunchKernelGGL(scan_kernel<true>, dim3(1), dim3(1024), 0, s, st, ca.TK, sa.TOFF, ca.TQ,
                           ca.TE, ca.HIST);
        GM_HIP(hipGetLastError());
      }
      hipLaunchKernelGGL(scatter_fn(d), dim3(scatter_grid_for(nb)), dim3(kTileThreads), 0, s, sa);
      GM_HIP(hipGetLastError());
      if (phases) GM_HIP(hipEventRecord(ev[k][4], s));
      nb = std::min<int64_t>(cap, 2 * nb);
    }
    GM_HIP(hipMemcpyAsync(pin ? (void*)pin : (void*)&hst, st, sizeof hst, hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    if (pin) hst = *pin;
    const int ran = (int)std::min<int64_t>(K, hst.iter - iter_done);
    if (ran <= 0 && !hst.done) {
      // the status block did not advance: never loop on it
      g_hip_err = "internal error: the device loop made no progress";
      return GM_EHIP;
    }
    iter_done = hst.iter;
    if (timing) {
      for (int k = 0; k < ran; ++k) {
        float a = 0, b = 0, c = 0, e = 0;
        GM_HIP(hipEventElapsedTime(&a, ev[k][0], ev[k][1]));
        if (phases) {
          GM_HIP(hipEventElapsedTime(&b, ev[k][1], ev[k][2]));
          GM_HIP(hipEventElapsedTime(&c, ev[k][2], ev[k][3]));
          GM_HIP(hipEventElapsedTime(&e, ev[k][3], ev[k][4]));
        }
        g_stats.rule_ms += a;
        g_stats.reduce_ms += b;
        g_stats.classify_ms += c;
        g_stats.split_ms += e;
        g_stats.rule_launches += 1;
      }
    }
    if (g_opt.log)
      std::fprintf(stderr, "gm: iter %lld n %lld I %.17g E %.6g T %.6g done %lld\n",
                   (long long)hst.iter, (long long)hst.n_active, hst.I, hst.E, hst.T,
                   (long long)hst.done);
    leaves_have = hst.leaf_count;
    if (hst.done) break;
    n = hst.n_active;
  }
  if (timing)
    for (auto& row : ev)
      for (auto& e : row) (void)hipEventDestroy(e);

  out->I = hst.I;
  out->E = hst.E;
  out->status = (int)hst.status;
  out->final_n = hst.n_active;
  out->final_npar = hst.n_par;
  out->final_split = hst.split;
  out->buf = hst.buf;
  out->leaf_count = keep_leaves ? hst.leaf_count : 0;
  out->base = base;
  out->lay = lay;
  out->cap = cap;
  out->vol_omega = vol;
  g_stats.iterations = hst.iter;
  g_stats.regions_evaluated = hst.regions_evaluated;
  g_stats.evals = hst.regions_evaluated * nodes_per_region(d);
  g_stats.max_active = hst.max_active;
  g_stats.final_active = hst.n_active;
  g_stats.finished = hst.finished;
  g_stats.status = hst.status;
  g_stats.total_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  g_last.valid = true;
  g_last.base = base;
  g_last.d = d;
  g_last.n = hst.n_active;
  g_last.npar = hst.n_par;
  g_last.split = hst.split;
  g_last.cap = cap;
  g_last.lay = lay;
  g_last.buf = hst.buf;
  return GM_OK;
}

}  // namespace gm

using namespace gm;

extern "C" {

int64_t gm_num_nodes(int d) {
  if (d < 1 || d > 62) return -1;
  return ((int64_t)1 << d) + 2 * (int64_t)d * d + 2 * (int64_t)d + 1;
}

int gm_integrate(int integrand_id, const double* params, int d, const double* lo, const double* hi,
                 double rel_tol, double abs_tol, int64_t max_regions, double* out_est,
                 double* out_err, void* stream) {
  int rc = validate(integrand_id, params, d, lo, hi, rel_tol, abs_tol);
  if (rc != GM_OK) return rc;
  if (!out_est || !out_err) return GM_EINVAL;
  std::lock_guard<std::mutex> lk(api_mutex());
  RunResult rr;
  rc = check_bounds(run_adaptive(integrand_id, params, d, lo, hi, rel_tol, abs_tol, max_regions,
                                 (hipStream_t)stream, false, &rr));
  if (rc != GM_OK) return rc;
  *out_est = rr.I;
  *out_err = rr.E;
  return rr.status;
}

int gm_integrate_noalloc(int integrand_id, const double* params, int d, const double* lo,
                         const double* hi, double rel_tol, double abs_tol, int64_t max_regions,
                         double* out_est, double* out_err, void* stream) {
  int rc = validate(integrand_id, params, d, lo, hi, rel_tol, abs_tol);
  if (rc != GM_OK) return rc;
  if (!out_est || !out_err || max_regions < 1) return GM_EINVAL;
  if (make_layout(d, max_regions).total > kNoallocScratchBytes) return GM_EINVAL;
  std::lock_guard<std::mutex> lk(api_mutex());
  char* base = nullptr;
  rc = noalloc_scratch(&base);
  if (rc != GM_OK) return rc;
  RunResult rr;
  rc = check_bounds(run_adaptive(integrand_id, params, d, lo, hi, rel_tol, abs_tol, max_regions,
                                 (hipStream_t)stream, false, &rr, base));
  if (rc != GM_OK) return rc;
  *out_est = rr.I;
  *out_err = rr.E;
  return rr.status;
}

int gm_eval_regions(int integrand_id, const double* params, int d, const double* lo,
                    const double* hi, int64_t n, const double* c, const double* h,
                    const int32_t* lvl, double* out_q, double* out_err, int32_t* out_axis,
                    void* stream) {
  int rc = validate(integrand_id, params, d, lo, hi, 1.0, 1.0);
  if (rc != GM_OK) return rc;
  if (n < 0 || (n > 0 && (!c || !h || !lvl || !out_q || !out_err || !out_axis))) return GM_EINVAL;
  for (int64_t r = 0; r < n; ++r)
    if (lvl[r] < 0 || lvl[r] > 65535) return GM_EINVAL;
  if (n == 0) return GM_OK;
  std::lock_guard<std::mutex> lk(api_mutex());
  hipStream_t s = (hipStream_t)stream;
  const int64_t cap = n;
  const Layout lay = make_layout(d, cap);
  char* base = nullptr;
  g_last.valid = false;  // (before the workspace may move)
  rc = acquire_workspace(lay.total, &base);
  if (rc != GM_OK) return rc;
  std::vector<double> cs((size_t)d * n), hs((size_t)d * n);
  std::vector<uint16_t> ls((size_t)n);
  for (int64_t r = 0; r < n; ++r) {
    for (int j = 0; j < d; ++j) {
      cs[(size_t)j * n + r] = c[r * d + j];
      hs[(size_t)j * n + r] = h[r * d + j];
    }
    ls[r] = (uint16_t)lvl[r];
  }
  RuleArgs ra;
  std::memset(&ra, 0, sizeof ra);
  fill_params(integrand_id, d, params, ra.P);
  fill_consts(d, ra.K);
  ra.C[0] = ra.C[1] = (const double*)(base + lay.C[0]);
  ra.H[0] = ra.H[1] = (const double*)(base + lay.H[0]);
  ra.L[0] = ra.L[1] = (const uint16_t*)(base + lay.L[0]);
  ra.cap = cap;
  ra.Q = (double*)(base + lay.Q);
  ra.ERR = (double*)(base + lay.ERR);
  ra.AXIS = (uint8_t*)(base + lay.AXIS);
  ra.partials = (double*)(base + lay.PART);
  ra.st = (Status*)(base + lay.ST);
  double vol = 1.0;
  for (int j = 0; j < d; ++j) vol = vol * (hi[j] - lo[j]);
  ra.vol_omega = vol;
  ra.n_fixed = n;
  GM_HIP(hipMemcpyAsync((void*)ra.C[0], cs.data(), sizeof(double) * d * n, hipMemcpyHostToDevice, s));
  GM_HIP(hipMemcpyAsync((void*)ra.H[0], hs.data(), sizeof(double) * d * n, hipMemcpyHostToDevice, s));
  GM_HIP(hipMemcpyAsync((void*)ra.L[0], ls.data(), sizeof(uint16_t) * n, hipMemcpyHostToDevice, s));
  const int map = choose_mapping(d, n);
  GM_HIP(launch_rule(d, integrand_id, map, ra, rule_grid(map, n, d), s));
  std::vector<uint8_t> ax((size_t)n);
  GM_HIP(hipMemcpyAsync(out_q, ra.Q, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  GM_HIP(hipMemcpyAsync(out_err, ra.ERR, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  GM_HIP(hipMemcpyAsync(ax.data(), ra.AXIS, n, hipMemcpyDeviceToHost, s));
  GM_HIP(hipStreamSynchronize(s));
  rc = check_bounds(GM_OK);
  if (rc != GM_OK) return rc;
  for (int64_t r = 0; r < n; ++r) out_axis[r] = ax[r];
  return GM_OK;
}

int64_t gm_last_active(int64_t offset, int64_t n, double* c, double* h, int32_t* lvl, double* q,
                       double* err, int32_t* axis) {
  std::lock_guard<std::mutex> lk(api_mutex());
  if (!g_last.valid) return 0;
  if (offset < 0) return GM_EINVAL;
  char* base = g_last.base;
  const int64_t cnt = std::min<int64_t>(n, g_last.n - offset);
  const int d = g_last.d;
  const int b = g_last.buf;
  const Layout& L = g_last.lay;
  if (cnt <= 0) return g_last.n;
  // Stored records behind regions [offset, offset + cnt): the same records when
  // the set is not split, else the records r mod n_par (one or two ranges).
  const bool split = g_last.split != 0;
  const int64_t npar = g_last.npar;
  auto rec = [&](int64_t r) { return (split && r >= npar) ? r - npar : r; };
  int64_t q0 = rec(offset), q1 = rec(offset + cnt - 1);
  if (split && offset < npar && offset + cnt > npar) {  // the window holds "-" and "+" children
    q0 = 0;
    q1 = npar - 1;
  }
  const int64_t nq = q1 - q0 + 1;
  std::vector<double> pc((size_t)nq * d), ph((size_t)nq * d);
  std::vector<uint16_t> pl((size_t)nq);
  std::vector<uint8_t> pa((size_t)nq, 0);
  for (int j = 0; j < d; ++j) {
    if (hipMemcpy(pc.data() + (size_t)j * nq, base + L.C[b] + sizeof(double) * (j * g_last.cap + q0),
                  sizeof(double) * nq, hipMemcpyDeviceToHost) != hipSuccess)
      return hip_fail(hipGetLastError());
    if (hipMemcpy(ph.data() + (size_t)j * nq, base + L.H[b] + sizeof(double) * (j * g_last.cap + q0),
                  sizeof(double) * nq, hipMemcpyDeviceToHost) != hipSuccess)
      return hip_fail(hipGetLastError());
  }
  if (hipMemcpy(pl.data(), base + L.L[b] + sizeof(uint16_t) * q0, sizeof(uint16_t) * nq,
                hipMemcpyDeviceToHost) != hipSuccess)
    return hip_fail(hipGetLastError());
  if (split && hipMemcpy(pa.data(), base + L.PAX[b] + q0, nq, hipMemcpyDeviceToHost) != hipSuccess)
    return hip_fail(hipGetLastError());
  for (int64_t i = 0; i < cnt; ++i) {
    const int64_t r = offset + i;
    const int64_t k = rec(r) - q0;
    const bool plus = split && r >= npar;
    const int ax = pa[k];
    for (int j = 0; j < d; ++j) {
      double cj = pc[(size_t)j * nq + k], hj = ph[(size_t)j * nq + k];
      if (split && j == ax) {  // the split of the Sec. 3 loop, as the device applies it
        const double hp = hj * 0.5;
        cj = plus ? cj + hp : cj - hp;
        hj = hp;
      }
      if (c) c[i * d + j] = cj;
      if (h) h[i * d + j] = hj;
    }
    if (lvl) lvl[i] = pl[k] + (split ? 1 : 0);
  }
  const size_t o8 = sizeof(double) * (size_t)offset;
  if (q && hipMemcpy(q, base + L.Q + o8, sizeof(double) * cnt, hipMemcpyDeviceToHost) != hipSuccess)
    return hip_fail(hipGetLastError());
  if (err &&
      hipMemcpy(err, base + L.ERR + o8, sizeof(double) * cnt, hipMemcpyDeviceToHost) != hipSuccess)
    return hip_fail(hipGetLastError());
  if (axis) {
    std::vector<uint8_t> a((size_t)cnt);
    if (hipMemcpy(a.data(), base + L.AXIS + offset, cnt, hipMemcpyDeviceToHost) != hipSuccess)
      return hip_fail(hipGetLastError());
    for (int64_t r = 0; r < cnt; ++r) axis[r] = a[r];
  }
  return g_last.n;
}

int gm_set_workspace(void* device_ptr, size_t bytes) {
  std::lock_guard<std::mutex> lk(api_mutex());
  g_last.valid = false;
  if (!device_ptr || bytes == 0) {
    g_ext_ptr = nullptr;
    g_ext_bytes = 0;
    return GM_OK;
  }
  if (((uintptr_t)device_ptr & 255u) != 0) return GM_EINVAL;
  g_ext_ptr = device_ptr;
  g_ext_bytes = bytes;
  return GM_OK;
}

size_t gm_workspace_bytes(int d, int64_t max_regions, int mode) {
  if (d < kMinDim || d > kMaxDim || max_regions < 1) return 0;
  if (mode == 2) return batch_layout_bytes(d, max_regions);
  return make_layout(d, max_regions).total;
}

int gm_set_option(const char* key, int64_t value) {
  if (!key) return GM_EINVAL;
  std::lock_guard<std::mutex> lk(api_mutex());
  const std::string k(key);
#ifdef GM_CHECK
  // (GM_CHECK builds only) "check_selftest" = n: a kernel checks index n
  // against bound n without accessing memory; the call returns what the
  // bounds-check path makes of it (GM_EHIP, the violation in
  // gm_status_string(GM_EHIP)).
  if (k == "check_selftest") {
    hipLaunchKernelGGL(check_selftest_kernel, dim3(1), dim3(64), 0, 0, value);
    GM_HIP(hipGetLastError());
    GM_HIP(hipDeviceSynchronize());
    return check_bounds(GM_OK);
  }
#endif
  if (k == "init_log2_regions") {
    if (value < 0 || value > 30) return GM_EINVAL;
    g_opt.init_log2 = (int)value;
  } else if (k == "max_iters") {
    if (value < 1 || value > 1000000) return GM_EINVAL;
    g_opt.max_iters = value;
  } else if (k == "graph_iters") {
    if (value < 0 || value > 64) return GM_EINVAL;
    g_opt.graph_iters = (int)value;
  } else if (k == "lanes_per_region") {
    if (value < 0 || value > 64 || (value & (value - 1))) return GM_EINVAL;
    g_opt.lanes_per_region = (int)value;
  } else if (k == "timing") {
    if (value < 0 || value > 2) return GM_EINVAL;
    g_opt.timing = (int)value;
  } else if (k == "rule") {
    if (value < 0 || value > 2) return GM_EINVAL;
    g_opt.rule = (int)value;
  } else if (k == "err_model") {
    if (value < 0 || value > 1) return GM_EINVAL;
    g_opt.err_model = (int)value;
  } else if (k == "prune") {
    if (value < 0 || value > 1) return GM_EINVAL;
    g_opt.prune = (int)value;
  } else if (k == "log") {
    g_opt.log = value ? 1 : 0;
  } else {
    return GM_EINVAL;
  }
  return GM_OK;
}

const char* gm_status_string(int status) {
  switch (status) {
    case GM_OK: return "converged: E <= max(abs_tol, rel_tol*|I|)";
    case GM_MAX_REGIONS: return "stopped: region capacity reached";
    case GM_MAX_ITERS: return "stopped: iteration budget used up";
    case GM_PRECISION_LIMIT: return "stopped: every region retired by a numerical guard, E > T";
    case GM_NONFINITE: return "integrand or a rule sum was not finite";
    case GM_EINVAL: return "invalid argument";
    case GM_ENOMEM:
      g_enomem_text = "out of device memory (or workspace too small); last HIP error: " + g_hip_err;
      return g_enomem_text.c_str();
    case GM_EHIP: return g_hip_err.c_str();
    default: return "unknown status";
  }
}

int gm_last_stats(gm_stats* out) {
  if (!out) return GM_EINVAL;
  std::lock_guard<std::mutex> lk(api_mutex());
  *out = g_stats;
  return GM_OK;
}

}  // extern "C"
