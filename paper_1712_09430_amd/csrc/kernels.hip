// HIP kernels (gfx950, wave64) of the sector-tracking hot path.
//
// Paper: arXiv:1712.09430, Sec. 2 item 1 (cellular-automaton seeding: links
// between hits of adjacent pad rows, seeds of at least three hits oriented
// along x) and item 2 (track following: fit the seed, extrapolate row by row,
// take the closest cluster per row, refine with a simplified Kalman filter in
// a constant field); Fig. 2 c-d; Tab. 1 rows 1-2.
//
// Floating point: compiled with -ffp-contract=off and without fast-math, so
// every float operation below is one IEEE binary32 operation rounded to
// nearest, in the order written (division and square root correctly
// rounded).  The operation order of the filter is part of the method's
// definition here: a different order would change results in the last bit and
// with them the hits that the gates accept.
//
// Layout and stage chain, for the sectors [s0, s1) of one call:
//   row index   per (sector, row): first hit of each row (binary search);
//               per hit: row range and order validation
//   grid        one wave per (sector, row): bounding box, bins, counting
//               sort of the row's hits into bin order (SortedHit)
//   neighbours  one thread per hit: best (up, down) pair in rows r+-1
//   clean/start one thread per hit: mutual links, start-hit bit (ballot)
//   scan        one workgroup: exclusive scan of per-block start counts
//   compact     one thread per hit: start list, per-sector tracklet offsets
//   tracklets   persistent, one lane per tracklet: seed chain, outward
//               following, back-transport, inward following
//   refit64     one lane per tracklet needing it: binary64-covariance refit
#include <float.h>

#include <algorithm>
#include <hip/hip_runtime.h>

#include "internal.h"

namespace catpc {
namespace {

__device__ __forceinline__ int sector_of(const int64_t* off, int s0, int s1, int64_t i) {
  // largest s in [s0, s1) with off[s] <= i  (off[s0] <= i < off[s1])
  int lo = s0, hi = s1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// Sector of hit i, walking forward from sector s (off[s] <= i, s < s1).
__device__ __forceinline__ int sector_from(const int64_t* off, int s1, int s, int64_t i) {
  while (s + 1 < s1 && off[s + 1] <= i) ++s;
  return s;
}

// Bin of a coordinate: monotone non-decreasing in v, clamped to [0, n-1].
__device__ __forceinline__ int bin_of(float v, float vmin, float inv, int n) {
  float f = (v - vmin) * inv;
  f = fminf(fmaxf(f, 0.0f), (float)(n - 1));
  return (int)f;
}

struct RowGrid {
  float ymin, zmin, iby, ibz;
  int ny, nz;
  const int32_t* bins;
  const SortedHit* hits;
};

// ------------------------------------------------------------------- reset
__global__ void k_reset(unsigned long long* c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0ull;
}

// Per-row neighbour-finder ratios from the pad-row planes on the device, each
// one binary32 division (the same values the host computes for a context):
// rowk[r] = (x_{r+1}/x_r, x_{r-1}/x_r, (x_r - x_{r-1}) / (x_{r+1} - x_{r-1}),
// x_r) for 1 <= r <= R-2, (0, 0, 0, x_r) otherwise.  Planes that are not
// positive and strictly ascending set error bit 6.
__global__ void k_rowk(const float* __restrict__ row_x, int R, float4* __restrict__ rowk,
                       unsigned long long* counters) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const float xr = row_x[r];
  float4 v = make_float4(0.0f, 0.0f, 0.0f, xr);
  if (r >= 1 && r + 1 < R) {
    const float xu = row_x[r + 1], xd = row_x[r - 1];
    v.x = xu / xr;
    v.y = xd / xr;
    v.z = (xr - xd) / (xu - xd);
  }
  rowk[r] = v;
  if (!(xr > 0.0f) || (r > 0 && !(xr > row_x[r - 1]))) atomicOr(&counters[kCtrError], 64ull);
}

// Copy of the error word of the chain (kCtrError) to the caller.
__global__ void k_status(const unsigned long long* counters, uint64_t* status) {
  if (threadIdx.x == 0) *status = counters[kCtrError];
}

// --------------------------------------------------------------- row index
// Blocks [0, item_blocks): one thread per (sector, row 0..R) item, first hit
// of the row by binary search (monotone in r for any input; row 0 starts at
// the sector's first hit and row R at its end, so the rows always partition
// the sector); the items of a sector also record it as the sector of the
// kHitsPerBlock-hit blocks that start in it, for the per-hit kernels after the
// neighbour search.  Remaining blocks: one thread per hit, order and range
// check.
__global__ __launch_bounds__(256) void k_row_index(Inputs in, Span sp, int R, const float* __restrict__ row_x,
                                                   int32_t* row_first, int32_t* blk_sec,
                                                   unsigned long long* counters, int64_t n_items,
                                                   int64_t item_blocks) {
  if ((int64_t)blockIdx.x < item_blocks) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_items) return;
    const int s = sp.s0 + (int)(g / (R + 1));
    const int r = (int)(g % (R + 1));
    const int64_t a = in.hit_offset[s], b = in.hit_offset[s + 1];
    // blocks whose first hit sp.h0 + k * kHitsPerBlock lies in [a, b)
    const int64_t k0 = (a - sp.h0 + kHitsPerBlock - 1) / kHitsPerBlock, k1 = (b - sp.h0 + kHitsPerBlock - 1) / kHitsPerBlock;
    for (int64_t k = k0 + r; k < k1; k += R + 1) blk_sec[k] = s;
    int64_t lo = a, hi = b;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (in.row[mid] < r) lo = mid + 1; else hi = mid;
    }
    row_first[(int64_t)s * (R + 1) + r] = (int32_t)((r == R ? b : r == 0 ? a : lo) - a);
  } else {
    const int64_t i = sp.h0 + ((int64_t)blockIdx.x - item_blocks) * blockDim.x + threadIdx.x;
    if (i < sp.h1) {
      const int32_t r = in.row[i];
      bool ok = r >= 0 && r < R;
      if (ok && i > sp.h0 && in.row[i - 1] > r) {
        // rows may fall only where a sector starts (rare: look the sector up then)
        const int s = sector_of(in.hit_offset, sp.s0, sp.s1, i);
        ok = in.hit_offset[s] == i;
      }
      if (!ok) atomicOr(&counters[kCtrError], 1ull);
      if (ok && in.x && !(in.x[i] == row_x[r])) atomicOr(&counters[kCtrError], 8ull);
    }
  }
}

// -------------------------------------------------------------------- grid
// Wave minimum / maximum of a float (all 64 lanes active; NaN not expected):
// floats as order-preserving integer keys, reduced inside each row of 16
// lanes by DPP moves (quad swaps, half-row and row mirrors), then the four
// row results read out.  Only the grid shape depends on these values.
__device__ __forceinline__ int float_key(float v) {
  const int b = __float_as_int(v);
  return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float key_float(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }

template <bool kMax>
__device__ __forceinline__ int wave_reduce_key(int v) {
  auto op = [](int x, int y) { return kMax ? max(x, y) : min(x, y); };
  v = op(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // lanes 1 0 3 2 of each quad
  v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // lanes 2 3 0 1 of each quad
  v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));  // mirror inside each half row
  v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));  // mirror inside each row
  const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
  const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
  return op(op(r0, r1), op(r2, r3));
}
__device__ __forceinline__ float wave_min(float v) { return key_float(wave_reduce_key<false>(float_key(v))); }
__device__ __forceinline__ float wave_max(float v) { return key_float(wave_reduce_key<true>(float_key(v))); }

constexpr int kGridKeep = 4;  // 64-hit rounds of a row kept in registers by the grid build

__global__ __launch_bounds__(64) void k_grid(Inputs in, Span sp, int R, float bin_hits, Workspace ws) {
  __shared__ int cnt[kMaxBinsPerRow];
  const int item = blockIdx.x;
  const int s = sp.s0 + item / R;
  const int r = item % R;
  const int lane = threadIdx.x;
  const int64_t gid = (int64_t)s * R + r;
  const int64_t a = in.hit_offset[s];
  const int32_t f0 = ws.row_first[(int64_t)s * (R + 1) + r];
  const int32_t f1 = ws.row_first[(int64_t)s * (R + 1) + r + 1];
  const int n = f1 - f0;
  const int64_t g = a + f0;
  if (n <= 0) {
    if (lane == 0) {
      RowHdr h = {0.0f, 0.0f, 0.0f, 0.0f, 0, 0, (int32_t)g, (int32_t)(g + gid), 0};
      ws.hdr[gid] = h;
    }
    return;
  }
  // the row's first kGridKeep * 64 hits stay in registers across the three
  // passes (range, count, scatter); the rest are read again
  float cy[kGridKeep], cz[kGridKeep];
  int cb[kGridKeep];
  float ylo = FLT_MAX, yhi = -FLT_MAX, zlo = FLT_MAX, zhi = -FLT_MAX;
#pragma unroll
  for (int q = 0; q < kGridKeep; ++q) {
    const int k = lane + 64 * q;
    cy[q] = 0.0f;
    cz[q] = 0.0f;
    if (k < n) {
      cy[q] = in.y[g + k];
      cz[q] = in.z[g + k];
      ylo = fminf(ylo, cy[q]); yhi = fmaxf(yhi, cy[q]);
      zlo = fminf(zlo, cz[q]); zhi = fmaxf(zhi, cz[q]);
    }
  }
  for (int k = lane + 64 * kGridKeep; k < n; k += 64) {
    const float y = in.y[g + k], z = in.z[g + k];
    ylo = fminf(ylo, y); yhi = fmaxf(yhi, y);
    zlo = fminf(zlo, z); zhi = fmaxf(zhi, z);
  }
  ylo = wave_min(ylo); yhi = wave_max(yhi);
  zlo = wave_min(zlo); zhi = wave_max(zhi);
  // grid shape: only the searches' speed depends on it (they test windows
  // exactly and take bin ranges with a margin), so hardware reciprocal and
  // square root are used here
  const int cap = min(2 * n + 1, kMaxBinsPerRow);
  int target = (int)fminf(ceilf((float)n * __builtin_amdgcn_rcpf(bin_hits)), (float)cap);
  target = max(target, 1);
  const float Ly = yhi - ylo, Lz = zhi - zlo;
  int ny = 1, nz = 1;
  if (Ly > 0.0f && Lz > 0.0f) {
    const float iw = __builtin_amdgcn_rsqf(Ly * Lz * __builtin_amdgcn_rcpf((float)target));
    ny = (int)fminf(ceilf(Ly * iw), (float)target);
    nz = (int)fminf(ceilf(Lz * iw), (float)target);
  } else if (Ly > 0.0f) {
    ny = target;
  } else if (Lz > 0.0f) {
    nz = target;
  }
  ny = max(ny, 1);
  nz = max(nz, 1);
  if (ny * nz > cap) {
    if (ny >= nz) ny = max(1, cap / nz); else nz = max(1, cap / ny);
  }
  const float iby = Ly > 0.0f ? (float)ny * __builtin_amdgcn_rcpf(Ly) : 0.0f;
  const float ibz = Lz > 0.0f ? (float)nz * __builtin_amdgcn_rcpf(Lz) : 0.0f;
  const float ymin = Ly > 0.0f ? ylo : 0.0f;
  const float zmin = Lz > 0.0f ? zlo : 0.0f;
  const int nb = ny * nz;
  if (lane == 0) {
    RowHdr h = {ymin, zmin, iby, ibz, (int16_t)ny, (int16_t)nz, (int32_t)g, (int32_t)(g + gid), n};
    ws.hdr[gid] = h;
  }
  for (int k = lane; k < nb; k += 64) cnt[k] = 0;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kGridKeep; ++q) {
    cb[q] = 0;
    if (lane + 64 * q < n) {
      cb[q] = bin_of(cz[q], zmin, ibz, nz) * ny + bin_of(cy[q], ymin, iby, ny);
      atomicAdd(&cnt[cb[q]], 1);
    }
  }
  for (int k = lane + 64 * kGridKeep; k < n; k += 64) {
    const int b = bin_of(in.z[g + k], zmin, ibz, nz) * ny + bin_of(in.y[g + k], ymin, iby, ny);
    atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  // exclusive scan of cnt[0, nb): each lane owns a contiguous slice
  const int per = (nb + 63) / 64;
  const int b0 = min(nb, lane * per), b1 = min(nb, b0 + per);
  int sum = 0;
  for (int b = b0; b < b1; ++b) sum += cnt[b];
  int incl = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o);
    if (lane >= o) incl += v;
  }
  int run = incl - sum;
  int32_t* bins = ws.bins + 2 * g + 2 * gid;
  for (int b = b0; b < b1; ++b) {
    const int c = cnt[b];
    bins[b] = run;
    cnt[b] = run;
    run += c;
  }
  if (lane == 0) bins[nb] = n;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kGridKeep; ++q) {
    const int k = lane + 64 * q;
    if (k < n) {
      const int pos = atomicAdd(&cnt[cb[q]], 1);
      SortedHit h;
      h.y = cy[q]; h.z = cz[q]; h.idx = f0 + k; h.row = r;
      ws.sorted[g + pos] = h;
    }
  }
  for (int k = lane + 64 * kGridKeep; k < n; k += 64) {
    const float y = in.y[g + k], z = in.z[g + k];
    const int b = bin_of(z, zmin, ibz, nz) * ny + bin_of(y, ymin, iby, ny);
    const int pos = atomicAdd(&cnt[b], 1);
    SortedHit h;
    h.y = y; h.z = z; h.idx = f0 + k; h.row = r;
    ws.sorted[g + pos] = h;
  }
}

// Global-to-LDS copies (global_load_lds): lane j of a copy instruction writes
// entry j of its (wave-uniform) LDS destination; nothing orders a later LDS
// read after them but a wait for the wave's memory operations.
typedef __attribute__((address_space(1))) void* GlobalPtr;
typedef __attribute__((address_space(3))) void* LdsPtr;

// Wait for the wave's outstanding global memory operations (the LDS copies
// among them: nothing else orders a later LDS read after them).
__device__ __forceinline__ void stage_wait() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), other counters not waited
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// --------------------------------------------------------------- neighbours
struct BinRange {
  int y0, y1, z0, z1;
};

__device__ __forceinline__ BinRange bin_range(const RowGrid& G, float yc, float wy, float zc, float wz) {
  BinRange b;
  b.y0 = bin_of((yc - wy) - kBinMargin, G.ymin, G.iby, G.ny);
  b.y1 = bin_of((yc + wy) + kBinMargin, G.ymin, G.iby, G.ny);
  b.z0 = bin_of((zc - wz) - kBinMargin, G.zmin, G.ibz, G.nz);
  b.z1 = bin_of((zc + wz) + kBinMargin, G.zmin, G.ibz, G.nz);
  return b;
}

// f(hit) for every hit in the bins [y0, y1] of the z rows [z0, z1] of G: the
// bin ranges of the first kFront rows are loaded together (one memory round
// trip instead of one per row) and hits are read two at a time.
template <int kFront, class F>
__device__ __forceinline__ void for_hits(const RowGrid& G, const BinRange& br, F&& f) {
  int ps[kFront], pe[kFront];
#pragma unroll
  for (int q = 0; q < kFront; ++q) {
    const int iz = min(br.z0 + q, br.z1);
    ps[q] = G.bins[iz * G.ny + br.y0];
    pe[q] = G.bins[iz * G.ny + br.y1 + 1];
    if (br.z0 + q > br.z1) pe[q] = ps[q];
  }
#pragma unroll
  for (int q = 0; q < kFront; ++q) {
    int p = ps[q];
    for (; p + 1 < pe[q]; p += 2) {
      const SortedHit h0 = G.hits[p], h1 = G.hits[p + 1];
      f(h0);
      f(h1);
    }
    if (p < pe[q]) f(G.hits[p]);
  }
  for (int iz = br.z0 + kFront; iz <= br.z1; ++iz) {
    const int e = G.bins[iz * G.ny + br.y1 + 1];
    for (int p = G.bins[iz * G.ny + br.y0]; p < e; ++p) f(G.hits[p]);
  }
}

constexpr int kNfKeep = 8;
constexpr int kNfMaxRows = 32;  // pad rows per neighbour-finder workgroup, at most

// Score the pair (up j, down k) for the hit (yi, zi) and keep the
// lexicographic minimum of (chi2, j, k) among pairs within the cut.
__device__ __forceinline__ void nf_consider(float yi, float zi, float t, float chi2max, float yj, float zj,
                                            int32_t j, float yk, float zk, int32_t k, float& best, int32_t& bj,
                                            int32_t& bk) {
  const float ey = yi - (yk + t * (yj - yk));
  const float ez = zi - (zk + t * (zj - zk));
  const float chi2 = ey * ey + ez * ez;
  if (!(chi2 <= chi2max)) return;
  if (bj < 0 || chi2 < best || (chi2 == best && (j < bj || (j == bj && k < bk)))) {
    best = chi2;
    bj = j;
    bk = k;
  }
}

// Grid of row rr of sector s, pointing into the LDS copy when the row is
// inside the staged range.
struct Stage {
  const RowHdr* hdr;      // LDS: headers of rows [r_lo, r_hi]
  const float4* rowk;     // LDS: rowk of rows [r_lo, r_hi]
  int r_lo, r_hi;         // staged rows [r_lo, r_hi]
  int64_t hit0, bin0;     // global sorted position / bin-table offset of the first staged row
  const SortedHit* hits;  // LDS
  const int32_t* bins;    // LDS
  bool on;
};

// kLds: every row the block reads is staged, and the pointers lead only to
// LDS, so the compiler emits LDS reads; otherwise they lead only to global
// memory.  (A pointer that may lead to either becomes a flat access, which
// is slower for both.)
template <bool kLds>
__device__ __forceinline__ RowGrid staged_grid(const Workspace& ws, int R, int s, int rr, const Stage& S) {
  const RowHdr h = S.hdr[rr - S.r_lo];
  RowGrid G;
  G.ymin = h.ymin; G.zmin = h.zmin; G.iby = h.iby; G.ibz = h.ibz;
  G.ny = h.ny;
  G.nz = h.nz;
  G.bins = ws.bins + 2 * (int64_t)h.bin_half;
  G.hits = ws.sorted + h.hit_base;
  (void)R;
  (void)s;  // the header comes from the block's LDS copy
  if (kLds) {
    G.hits = S.hits + (G.hits - (ws.sorted + S.hit0));
    G.bins = S.bins + (G.bins - (ws.bins + S.bin0));
  }
  return G;
}

// The neighbour search of the block's hits (`own`, n of them, grid order).
template <bool kLds>
__device__ __forceinline__ void nf_hits(const SortedHit* own, int n, int64_t a, int s, int R,
                                        const float4* __restrict__ rowk, const Consts& c, const Workspace& ws,
                                        const Stage& S, int32_t* __restrict__ out_up, int32_t* __restrict__ out_dn) {
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const SortedHit me = own[k];
    const int r = me.row;
    int32_t bj = -1, bk = -1;
    if (r >= 1 && r <= R - 2) {
      const RowGrid U = staged_grid<kLds>(ws, R, s, r + 1, S);
      const RowGrid D = staged_grid<kLds>(ws, R, s, r - 1, S);
      if (U.ny > 0 && D.ny > 0) {
        const float4 f = S.rowk[r - S.r_lo];
        const float fu = f.x, fd = f.y, t = f.z;
        const float yi = me.y, zi = me.z;
        const float yu = yi * fu, zu = zi * fu;
        const float yd = yi * fd, zd = zi * fd;
        const BinRange ru = bin_range(U, yu, c.wy, zu, c.wz);
        const BinRange rd = bin_range(D, yd, c.wy, zd, c.wz);
        float ky[kNfKeep], kz[kNfKeep];
        int32_t ki[kNfKeep];
        int nk = 0;
        bool spill = false;
        for (int jz = rd.z0; jz <= rd.z1; ++jz) {
          const int qe = D.bins[jz * D.ny + rd.y1 + 1];
          for (int q = D.bins[jz * D.ny + rd.y0]; q < qe; ++q) {
            const SortedHit hk = D.hits[q];
            if (!(fabsf(hk.y - yd) <= c.wy && fabsf(hk.z - zd) <= c.wz)) continue;
#pragma unroll
            for (int m = 0; m < kNfKeep; ++m)
              if (m == nk) { ky[m] = hk.y; kz[m] = hk.z; ki[m] = hk.idx; }
            spill = spill || nk == kNfKeep;
            nk = min(nk + 1, kNfKeep);
          }
        }
        float best = 0.0f;
        if (nk > 0) {
          for (int iz = ru.z0; iz <= ru.z1; ++iz) {
            const int pe = U.bins[iz * U.ny + ru.y1 + 1];
            for (int p = U.bins[iz * U.ny + ru.y0]; p < pe; ++p) {
              const SortedHit hj = U.hits[p];
              if (!(fabsf(hj.y - yu) <= c.wy && fabsf(hj.z - zu) <= c.wz)) continue;
              if (!spill) {
#pragma unroll
                for (int m = 0; m < kNfKeep; ++m)
                  if (m < nk) nf_consider(yi, zi, t, c.chi2, hj.y, hj.z, hj.idx, ky[m], kz[m], ki[m], best, bj, bk);
              } else {
                for (int jz = rd.z0; jz <= rd.z1; ++jz) {
                  const int qe = D.bins[jz * D.ny + rd.y1 + 1];
                  for (int q = D.bins[jz * D.ny + rd.y0]; q < qe; ++q) {
                    const SortedHit hk = D.hits[q];
                    if (!(fabsf(hk.y - yd) <= c.wy && fabsf(hk.z - zd) <= c.wz)) continue;
                    nf_consider(yi, zi, t, c.chi2, hj.y, hj.z, hj.idx, hk.y, hk.z, hk.idx, best, bj, bk);
                  }
                }
              }
            }
          }
        }
      }
    }
    const int64_t i = a + me.idx;
    out_up[i] = bj;
    out_dn[i] = bk;
  }
}

// One workgroup per (sector, chunk of `rows` pad rows); its lanes take the
// chunk's hits in grid order (all rows of the chunk together, so sparse rows
// do not leave lanes idle).  The chunk's rows and the row on each side are
// contiguous in the grid-sorted array and in the bin tables; they are staged
// in LDS when they fit in `lds_bytes` (dynamic shared memory), else read in
// place.  Down-row candidates inside the window are kept in registers (up to
// kNfKeep; beyond that the down row is scanned again per up candidate).  Hits
// of rows 0 and R-1 get -1 links.  rowk[r] = (x_{r+1}/x_r, x_{r-1}/x_r,
// (x_r - x_{r-1}) / (x_{r+1} - x_{r-1})), each one binary32 division.
__global__ __launch_bounds__(256) void k_neighbours(Inputs in, Span sp, int R, const float4* __restrict__ rowk,
                                                    Consts c, Workspace ws, int32_t* __restrict__ out_up,
                                                    int32_t* __restrict__ out_dn, int rows, int lds_bytes) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int chunks = (R + rows - 1) / rows;
  const int s = sp.s0 + (int)(blockIdx.x / chunks);
  const int c0 = (int)(blockIdx.x % chunks) * rows;
  const int c1 = min(R, c0 + rows);
  const int32_t* rf = ws.row_first + (int64_t)s * (R + 1);
  const int n = rf[c1] - rf[c0];
  if (n <= 0) return;
  const int64_t a = in.hit_offset[s];
  Stage S;
  S.on = false;
  S.r_lo = max(c0 - 1, 0);
  S.r_hi = min(c1, R - 1);
  // the rows' hits and bin tables are copied into LDS (global-to-LDS, no
  // registers: lane j of a copy writes entry j of its destination; each wave
  // takes every (blockDim/64)-th run of 64 entries) when they fit, issued
  // before the row headers are read so that one wait and one barrier cover both
  const int64_t h0 = a + rf[S.r_lo], h1 = a + rf[S.r_hi + 1];
  const int64_t b0 = 2 * (h0 + (int64_t)s * R + S.r_lo);
  const int64_t b1 = 2 * (h1 + (int64_t)s * R + S.r_hi + 1);
  const int64_t nh = h1 - h0, nb = b1 - b0;
  if (nh * (int64_t)sizeof(SortedHit) + nb * (int64_t)sizeof(int32_t) <= lds_bytes) {
    SortedHit* lh = reinterpret_cast<SortedHit*>(lds);
    int32_t* lb = reinterpret_cast<int32_t*>(lds + nh * sizeof(SortedHit));
    const int lane = threadIdx.x & 63;
    for (int64_t base = threadIdx.x - lane; base < nh; base += blockDim.x)
      if (base + lane < nh)
        __builtin_amdgcn_global_load_lds((GlobalPtr)(ws.sorted + h0 + base + lane), (LdsPtr)(lh + base), 16, 0, 0);
    for (int64_t base = threadIdx.x - lane; base < nb; base += blockDim.x)
      if (base + lane < nb)
        __builtin_amdgcn_global_load_lds((GlobalPtr)(ws.bins + b0 + base + lane), (LdsPtr)(lb + base), 4, 0, 0);
    S.on = true;
    S.hit0 = h0;
    S.bin0 = b0;
    S.hits = lh;
    S.bins = lb;
  }
  // row headers and row constants of the block's rows and their neighbours
  __shared__ RowHdr nf_hdr[kNfMaxRows + 2];
  __shared__ float4 nf_rowk[kNfMaxRows + 2];
  for (int k = threadIdx.x; k <= S.r_hi - S.r_lo; k += blockDim.x) {
    nf_hdr[k] = ws.hdr[(int64_t)s * R + S.r_lo + k];
    nf_rowk[k] = rowk[S.r_lo + k];
  }
  S.hdr = nf_hdr;
  S.rowk = nf_rowk;
  if (S.on) stage_wait();
  __syncthreads();
  if (S.on)
    nf_hits<true>(S.hits + (a + rf[c0] - S.hit0), n, a, s, R, rowk, c, ws, S, out_up, out_dn);
  else
    nf_hits<false>(ws.sorted + a + rf[c0], n, a, s, R, rowk, c, ws, S, out_up, out_dn);
}

// Renumbering of a launch's workgroups so that each die (workgroups are dealt
// out round-robin over the kXcds dies) takes one contiguous run of them: the
// neighbour rows that consecutive workgroups share stay in one die's L2.
__device__ __forceinline__ int64_t die_contiguous(int64_t b, int64_t nblk) {
  const int64_t x = b % kXcds, k = b / kXcds;
  const int64_t q = nblk / kXcds, rem = nblk % kXcds;
  return x * q + min(x, rem) + k;
}

// The hits of a window in one row of a bin grid: the ranges of its first two
// z rows of bins (loaded together), and the bounds of any further z row.
// Bin b of the row (b = z * ny + y) spans positions [cs[base + b],
// cs[base + b + 1]).
struct NfWin {
  int p0, n0, p1, n1;
  int y0, y1, z2, z1, base, ny;
};

__device__ __forceinline__ NfWin nf_window(const int32_t* cs, int base, float ymin, float iby, int ny, float zmin,
                                           float ibz, int nz, float yc, float wy, float zc, float wz) {
  NfWin w;
  w.y0 = bin_of((yc - wy) - kBinMargin, ymin, iby, ny);
  w.y1 = bin_of((yc + wy) + kBinMargin, ymin, iby, ny);
  const int z0 = bin_of((zc - wz) - kBinMargin, zmin, ibz, nz);
  w.z1 = bin_of((zc + wz) + kBinMargin, zmin, ibz, nz);
  w.base = base;
  w.ny = ny;
  const int r0 = w.base + z0 * ny;
  const int r1 = w.base + min(z0 + 1, w.z1) * ny;
  w.p0 = cs[r0 + w.y0];
  w.n0 = cs[r0 + w.y1 + 1] - w.p0;
  w.p1 = cs[r1 + w.y0];
  w.n1 = z0 < w.z1 ? cs[r1 + w.y1 + 1] - w.p1 : 0;
  w.z2 = z0 + 2;
  return w;
}

// f(position) for every hit position of the window: the first two z rows as
// one flat loop (lanes whose windows differ only in how the hits split over
// the two rows run the same number of iterations), then any further z row.
template <class F>
__device__ __forceinline__ void nf_for(const NfWin& w, const int32_t* cs, F&& f) {
  const int n = w.n0 + w.n1;
  for (int k = 0; k < n; ++k) f(k < w.n0 ? w.p0 + k : w.p1 + (k - w.n0));
  for (int iz = w.z2; iz <= w.z1; ++iz) {
    const int rr = w.base + iz * w.ny;
    const int e = cs[rr + w.y1 + 1];
    for (int p = cs[rr + w.y0]; p < e; ++p) f(p);
  }
}

// Keep the lexicographic minimum of (chi2, j, k) among pairs within the cut.
__device__ __forceinline__ void nf_keep(float chi2, float chi2max, int32_t j, int32_t k, float& best, int32_t& bj,
                                        int32_t& bk) {
  if (!(chi2 <= chi2max)) return;
  if (bj < 0 || chi2 < best || (chi2 == best && (j < bj || (j == bj && k < bk)))) {
    best = chi2;
    bj = j;
    bk = k;
  }
}

// Neighbour finder, in place.  One thread per hit in the order of the
// grid-sorted array (sector, pad row, bin), so the lanes of a wave take hits
// of one row and of the same or adjacent bins: their windows, and the number
// of candidates they visit, are alike.  For the hit in row r the down
// candidates (row r-1) and up candidates (row r+1) are the hits of the bins
// the +-wy x +-wz windows around the ray predictions y x_{r+-1}/x_r,
// z x_{r+-1}/x_r touch; every up candidate inside its window is paired with
// every down candidate inside its window, re-read from memory (no per-lane
// candidate list, so the kernel stays small enough for many resident waves).
// Workgroups are renumbered die-contiguously.  rowk[r] = (x_{r+1}/x_r,
// x_{r-1}/x_r, (x_r - x_{r-1}) / (x_{r+1} - x_{r-1})), each one binary32
// division.
__global__ __launch_bounds__(256) void k_nf_flat(Inputs in, Span sp, int R, const float4* __restrict__ rowk,
                                                 Consts c, Workspace ws, int32_t* __restrict__ out_up,
                                                 int32_t* __restrict__ out_dn, int64_t nblk) {
  const int64_t L = die_contiguous(blockIdx.x, nblk);
  const int64_t i = sp.h0 + L * blockDim.x + threadIdx.x;
  if (i >= sp.h1) return;
  const int64_t kb = (i - sp.h0) / kHitsPerBlock;
  const int s = sector_from(in.hit_offset, sp.s1, ws.blk_sec[kb], i);
  const SortedHit me = ws.sorted[i];
  const int r = me.row;
  const int64_t gr = (int64_t)s * R + r;
  int32_t bj = -1, bk = -1;
  if (r >= 1 && r <= R - 2) {
    const RowHdr hu = ws.hdr[gr + 1], hd = ws.hdr[gr - 1];
    if (hu.ny > 0 && hd.ny > 0) {
      const float4 f = rowk[r];
      const float fu = f.x, fd = f.y, t = f.z;
      const float yi = me.y, zi = me.z;
      const float yu = yi * fu, zu = zi * fu;
      const float yd = yi * fd, zd = zi * fd;
      const int32_t* bu = ws.bins + 2 * (int64_t)hu.bin_half;
      const int32_t* bd = ws.bins + 2 * (int64_t)hd.bin_half;
      const SortedHit* su = ws.sorted + hu.hit_base;
      const SortedHit* sd = ws.sorted + hd.hit_base;
      const NfWin wu = nf_window(bu, 0, hu.ymin, hu.iby, hu.ny, hu.zmin, hu.ibz, hu.nz, yu, c.wy, zu, c.wz);
      const NfWin wd = nf_window(bd, 0, hd.ymin, hd.iby, hd.ny, hd.zmin, hd.ibz, hd.nz, yd, c.wy, zd, c.wz);
      float best = 0.0f;
      nf_for(wu, bu, [&](int pj) {
        const float4 hj = *reinterpret_cast<const float4*>(su + pj);
        if (!(fabsf(hj.x - yu) <= c.wy && fabsf(hj.y - zu) <= c.wz)) return;
        const int32_t j = __float_as_int(hj.z);
        nf_for(wd, bd, [&](int pk) {
          const float4 hk = *reinterpret_cast<const float4*>(sd + pk);
          if (!(fabsf(hk.x - yd) <= c.wy && fabsf(hk.y - zd) <= c.wz)) return;
          const float ey = yi - (hk.x + t * (hj.x - hk.x));
          const float ez = zi - (hk.y + t * (hj.y - hk.y));
          nf_keep(ey * ey + ez * ez, c.chi2, j, __float_as_int(hk.z), best, bj, bk);
        });
      });
    }
  }
  const int64_t o = in.hit_offset[s] + me.idx;
  out_up[o] = bj;
  out_dn[o] = bk;
}

// -------------------------------------------------------------- clean/start
// One workgroup per kCleanRounds consecutive blocks of kHitsPerBlock hits:
// each thread takes one hit of every block, issuing the loads of all its hits
// before the gathers that depend on them (the kernel is bound by the latency
// of the chain hit -> link -> link of the linked hit).  Start bits, their
// per-block counts and every output keep the kHitsPerBlock blocking.
constexpr int kCleanRounds = 4;

__global__ __launch_bounds__(kHitsPerBlock) void k_clean_start(Inputs in, Span sp, int64_t nblk,
                                                               const int32_t* __restrict__ up,
                                                               const int32_t* __restrict__ dn,
                                                               int32_t* __restrict__ uc_out,
                                                               int32_t* __restrict__ dc_out, Workspace ws) {
  constexpr int K = kCleanRounds;
  const int64_t hb0 = (int64_t)blockIdx.x * K;
  int64_t i[K], a[K];
  int32_t u[K], d[K], uc[K], dc[K];
  float y[K], z[K];
  bool on[K], start[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    i[k] = sp.h0 + (hb0 + k) * kHitsPerBlock + threadIdx.x;
    on[k] = hb0 + k < nblk && i[k] < sp.h1;
    u[k] = -1; d[k] = -1; a[k] = 0; y[k] = 0.f; z[k] = 0.f;
    if (on[k]) {
      const int s = sector_from(in.hit_offset, sp.s1, ws.blk_sec[hb0 + k], i[k]);
      a[k] = in.hit_offset[s];
      u[k] = up[i[k]];
      d[k] = dn[i[k]];
      y[k] = in.y[i[k]];
      z[k] = in.z[i[k]];
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int32_t me = (int32_t)(i[k] - a[k]);
    uc[k] = (u[k] >= 0 && dn[a[k] + u[k]] == me) ? u[k] : -1;
    dc[k] = (d[k] >= 0 && up[a[k] + d[k]] == me) ? d[k] : -1;
  }
  int32_t w[K];
#pragma unroll
  for (int k = 0; k < K; ++k) w[k] = (dc[k] < 0 && uc[k] >= 0) ? up[a[k] + uc[k]] : -1;
#pragma unroll
  for (int k = 0; k < K; ++k) start[k] = w[k] >= 0 && dn[a[k] + w[k]] == uc[k];
  __shared__ int wc[K][kHitsPerBlock / 64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (on[k]) {
      uc_out[i[k]] = uc[k];
      dc_out[i[k]] = dc[k];
      ChainHit ch;
      ch.y = y[k];
      ch.z = z[k];
      ch.up = uc[k];
      ch.pad = 0;
      ws.chain[i[k]] = ch;
    }
    const unsigned long long m = __ballot(start[k]);
    if (lane == 0) {
      if (hb0 + k < nblk) ws.start_mask[(hb0 + k) * (kHitsPerBlock / 64) + wave] = m;
      wc[k][wave] = __popcll(m);
    }
  }
  __syncthreads();
  if (threadIdx.x < K && hb0 + threadIdx.x < nblk) {
    int t = 0;
    for (int v = 0; v < kHitsPerBlock / 64; ++v) t += wc[threadIdx.x][v];
    ws.blk_cnt[hb0 + threadIdx.x] = t;
  }
}

// -------------------------------------------------------------------- scan
// Two levels: each workgroup scans 1024 consecutive block counts (block
// offsets relative to the group), then one workgroup scans the group totals.
// The compaction adds the two.
constexpr int kScanGroup = 1024;

__global__ __launch_bounds__(kScanGroup) void k_scan_local(int64_t nblk, Workspace ws) {
  __shared__ int wsum[kScanGroup / 64];
  const int64_t b = (int64_t)blockIdx.x * kScanGroup + threadIdx.x;
  const int v = b < nblk ? ws.blk_cnt[b] : 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(incl, o);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    int x = lane < kScanGroup / 64 ? wsum[lane] : 0;
    for (int o = 1; o < kScanGroup / 64; o <<= 1) {
      const int u = __shfl_up(x, o);
      if (lane >= o) x += u;
    }
    if (lane < kScanGroup / 64) wsum[lane] = x;
  }
  __syncthreads();
  // entry nblk (one past the last block) gets the group's full prefix
  if (b <= nblk) ws.blk_off[b] = (wave ? wsum[wave - 1] : 0) + incl - v;
  if (threadIdx.x == kScanGroup - 1) ws.grp_off[blockIdx.x] = wsum[kScanGroup / 64 - 1];
}

// In-place exclusive scan of the ng group totals (plus the span's base slot);
// grp_off[ng] = end of the span's slots.  Also clears the tracklet kernel's
// work counters.
__global__ __launch_bounds__(1024) void k_scan_top(Span sp, int64_t ng, int64_t* toff, Workspace ws) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (ng + 1023) / 1024;
  const int64_t g0 = min(ng, (int64_t)t * per), g1 = min(ng, g0 + per);
  int64_t sum = 0;
  for (int64_t g = g0; g < g1; ++g) sum += ws.grp_off[g];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  const int64_t base = sp.s0 == 0 ? 0 : toff[sp.s0];
  int64_t run = base + part[t] - sum;
  for (int64_t g = g0; g < g1; ++g) {
    const int64_t v = ws.grp_off[g];
    ws.grp_off[g] = run;
    run += v;
  }
  if (t == 1023) ws.grp_off[ng] = base + part[1023];
  if (t == 0) {
    if (sp.s0 == 0) toff[0] = 0;
    for (int k = 0; k < kXcds; ++k) ws.counters[kCtrWork + k] = 0ull;
  }
}

__device__ __forceinline__ int64_t block_slot(const Workspace& ws, int64_t b) {
  return ws.grp_off[b / kScanGroup] + ws.blk_off[b];
}

// ----------------------------------------------------------------- compact
// Blocks [0, word_blocks): one thread per 64-hit word of the start mask; a
// word with start hits writes them in ascending order from its offset (the
// block offset plus the counts of the words before it in the block).  The
// remaining blocks: one thread per sector boundary, the sector's first slot.
__global__ __launch_bounds__(kHitsPerBlock) void k_compact(Inputs in, Span sp, int64_t nblk, int64_t word_blocks,
                                                           int64_t* toff, int32_t* __restrict__ start_hit,
                                                           Workspace ws) {
  constexpr int W = kHitsPerBlock / 64;  // mask words per clean/start block
  if ((int64_t)blockIdx.x < word_blocks) {
    const int64_t g = (int64_t)blockIdx.x * kHitsPerBlock + threadIdx.x;  // mask word
    const int64_t i0 = sp.h0 + g * 64;
    unsigned long long m = g < nblk * W ? ws.start_mask[g] : 0ull;  // no bits past the span's last hit
    if (m) {
      const int64_t b = g / W;
      int s = ws.blk_sec[b];
      int64_t pos = block_slot(ws, b);
      for (int64_t w = b * W; w < g; ++w) pos += __popcll(ws.start_mask[w]);
      do {
        const int64_t i = i0 + (__ffsll((long long)m) - 1);
        while (s + 1 < sp.s1 && in.hit_offset[s + 1] <= i) ++s;
        start_hit[pos] = (int32_t)(i - in.hit_offset[s]);
        ws.start_glob[pos] = (int32_t)i;
        ++pos;
        m &= m - 1ull;
      } while (m);
    }
  } else {
    const int s = sp.s0 + 1 + (int)(((int64_t)blockIdx.x - word_blocks) * kHitsPerBlock + threadIdx.x);
    if (s <= sp.s1) {
      const int64_t j = in.hit_offset[s] - sp.h0;
      const int64_t b = j / kHitsPerBlock;
      int64_t p = block_slot(ws, b);
      for (int64_t w = b * W; w < j / 64; ++w) p += __popcll(ws.start_mask[w]);
      const int rem = (int)(j & 63);
      if (rem) p += __popcll(ws.start_mask[j / 64] & ((1ull << rem) - 1ull));
      toff[s] = p;
    }
  }
}

// ------------------------------------------------------------ Kalman filter
struct Trk {
  float x, y, z, s, l, q;
  float c00, c10, c11, c20, c21, c22;
  float d00, d10, d11;
};

enum { kStepOk = 0, kStepSinPhi = 1, kStepArc = 2 };

__device__ __forceinline__ int init_track(Trk& t, float x0, float y0, float z0, float x1, float y1, float z1,
                                          const Consts& c) {
  const float dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
  const float L = sqrtf(dx * dx + dy * dy);
  t.x = x0; t.y = y0; t.z = z0;
  t.s = dy / L;
  t.l = dz / L;
  t.q = 0.0f;
  t.c00 = c.sy2; t.c10 = 0.0f; t.c11 = 1.0f; t.c20 = 0.0f; t.c21 = 0.0f; t.c22 = 100.0f;
  t.d00 = c.sz2; t.d10 = 0.0f; t.d11 = 1.0f;
  return fabsf(t.s) < 0.999f ? kStepOk : kStepSinPhi;
}

// Correctly rounded square root for binary32 x that is normal, finite and at
// least 2^-96: the hardware square root (within one ulp) and the choice
// between it and its two neighbours by the signs of the fused residuals
// x - s' s.  For such x these are the steps of the library's correctly
// rounded sqrtf (its range scaling and its special-value fix-up do not
// apply), so the result equals sqrtf(x) bit for bit; catpc_fp32_probe op 5
// exposes it so that this is checked over every such x.  Used where
// x = 1 - s^2 with |s| < 0.999, x in [0.001999, 1].
__device__ __forceinline__ float sqrt_unit(float x) {
  const float s = __builtin_amdgcn_sqrtf(x);
  const float dn = __int_as_float(__float_as_int(s) - 1);
  const float up = __int_as_float(__float_as_int(s) + 1);
  const float r_dn = __builtin_fmaf(-dn, s, x);
  const float r_up = __builtin_fmaf(-up, s, x);
  float v = r_dn <= 0.0f ? dn : s;
  v = r_up > 0.0f ? up : v;
  return v;
}

// Helix transport to x1 (constant field): exact state transport, arc length
// from the asin(u)/u series through u^8, covariance C <- J C J^T per block.
__device__ __forceinline__ int propagate(Trk& t, float x1, const Consts& c) {
  const float dx = x1 - t.x;
  const float k = c.kb * t.q;
  const float s0 = t.s;
  const float s1 = s0 + k * dx;
  if (!(fabsf(s1) < 0.999f)) return kStepSinPhi;
  // |s0|, |s1| < 0.999 (every state the transport sees passed that check)
  const float c0 = sqrt_unit(1.0f - s0 * s0);
  const float c1 = sqrt_unit(1.0f - s1 * s1);
  const float T = (s0 + s1) / (c0 + c1);
  const float dy = dx * T;
  const float ch = sqrtf(dx * dx + dy * dy);
  const float u = (k * ch) * 0.5f;
  if (!(fabsf(u) <= 0.2f)) return kStepArc;
  const float u2 = u * u;
  const float A = 1.0f + u2 * (1.0f / 6.0f + u2 * (3.0f / 40.0f + u2 * (5.0f / 112.0f + u2 * (35.0f / 1152.0f))));
  float dS = ch * A;
  if (dx < 0.0f) dS = -dS;
  const float sm = (s0 + s1) * 0.5f;
  const float cm2 = 1.0f - sm * sm;
  const float cm3 = cm2 * sqrt_unit(cm2);
  const float a = dx / cm3;
  const float b = ((c.kb * dx) * dx * 0.5f) / cm3;
  const float d = c.kb * dx;
  t.x = x1;
  t.y = t.y + dy;
  t.z = t.z + t.l * dS;
  t.s = s1;
  const float c00 = t.c00, c10 = t.c10, c11 = t.c11, c20 = t.c20, c21 = t.c21, c22 = t.c22;
  const float m0 = c00 + a * c10 + b * c20;
  const float m1 = c10 + a * c11 + b * c21;
  const float m2 = c20 + a * c21 + b * c22;
  const float n1 = c11 + d * c21;
  const float n2 = c21 + d * c22;
  t.c00 = m0 + a * m1 + b * m2;
  t.c10 = m1 + d * m2;
  t.c11 = n1 + d * n2;
  t.c20 = m2;
  t.c21 = n2;
  const float tz = t.d10 + dS * t.d11;
  t.d00 = t.d00 + dS * t.d10 + dS * tz;
  t.d10 = tz;
  return kStepOk;
}

// Kalman update with a cluster (my, mz): independent scalar updates of the
// transverse (y, s, q) and longitudinal (z, l) blocks.  An update that would
// take |sin phi| to 0.999 or beyond is rejected and leaves the state as it was.
__device__ __forceinline__ int update(Trk& t, float my, float mz, const Consts& c) {
  const float ry = my - t.y;
  const float Sy = t.c00 + c.sy2;
  const float iy = 1.0f / Sy;
  const float k0 = t.c00 * iy, k1 = t.c10 * iy, k2 = t.c20 * iy;
  const float s1 = t.s + k1 * ry;
  if (!(fabsf(s1) < 0.999f)) return kStepSinPhi;
  t.y = t.y + k0 * ry;
  t.s = s1;
  t.q = t.q + k2 * ry;
  const float c00 = t.c00, c10 = t.c10, c20 = t.c20;
  t.c00 = c00 - k0 * c00;
  t.c10 = c10 - k1 * c00;
  t.c20 = c20 - k2 * c00;
  t.c11 = t.c11 - k1 * c10;
  t.c21 = t.c21 - k2 * c10;
  t.c22 = t.c22 - k2 * c20;
  const float rz = mz - t.z;
  const float Sz = t.d00 + c.sz2;
  const float iz = 1.0f / Sz;
  const float g0 = t.d00 * iz, g1 = t.d10 * iz;
  t.z = t.z + g0 * rz;
  t.l = t.l + g1 * rz;
  const float d00 = t.d00, d10 = t.d10;
  t.d00 = d00 - g0 * d00;
  t.d10 = d10 - g1 * d00;
  t.d11 = t.d11 - g1 * d10;
  return kStepOk;
}

__device__ __forceinline__ bool spd_ok(const Trk& t) {
  const float p0 = t.c00;
  if (!(p0 > 0.0f && p0 <= FLT_MAX)) return false;
  const float i0 = 1.0f / p0;
  const float a = t.c10 * i0;
  const float p1 = t.c11 - a * t.c10;
  if (!(p1 > 0.0f && p1 <= FLT_MAX)) return false;
  const float b = t.c20 * i0;
  const float e = t.c21 - b * t.c10;
  const float g = e / p1;
  const float p2 = (t.c22 - b * t.c20) - g * e;
  if (!(p2 > 0.0f && p2 <= FLT_MAX)) return false;
  const float q0 = t.d00;
  if (!(q0 > 0.0f && q0 <= FLT_MAX)) return false;
  const float q1 = t.d11 - (t.d10 / q0) * t.d10;
  if (!(q1 > 0.0f && q1 <= FLT_MAX)) return false;
  return true;
}

struct Work {
  int n_prop, n_upd, n_cand, n_search;
};

// A cluster: sector-local index (-1: none) and its coordinates.
struct Pick {
  int32_t idx;
  float y, z;
};

constexpr int kClosestRows = 2;  // z rows of a search whose bin ranges are loaded up front

// Closest gated cluster of a row: smallest dy^2 + dz^2, ties to the smaller
// sector-local index.
__device__ __forceinline__ Pick closest(const Trk& t, const RowGrid& G, const Consts& c, Work& w) {
  const float gy = c.nsig * sqrtf(t.c00 + c.sy2);
  const float gz = c.nsig * sqrtf(t.d00 + c.sz2);
  Pick best = {-1, 0.0f, 0.0f};
  ++w.n_search;
  if (G.ny <= 0) return best;
  const BinRange br = bin_range(G, t.y, gy, t.z, gz);
  float bd = 0.0f;
  auto take = [&](const SortedHit& h) {
    const float dy = h.y - t.y;
    const float dz = h.z - t.z;
    if (!(fabsf(dy) <= gy && fabsf(dz) <= gz)) return;
    ++w.n_cand;
    const float d2 = dy * dy + dz * dz;
    if (best.idx < 0 || d2 < bd || (d2 == bd && h.idx < best.idx)) {
      best.idx = h.idx;
      best.y = h.y;
      best.z = h.z;
      bd = d2;
    }
  };
  // the result is the minimum of (d2, index) whatever the order of the hits
  for_hits<kClosestRows>(G, br, take);
  return best;
}

__device__ __forceinline__ RowGrid grid_of(const RowHdr& h, const Workspace& ws) {
  RowGrid G;
  G.ymin = h.ymin; G.zmin = h.zmin; G.iby = h.iby; G.ibz = h.ibz;
  G.ny = h.ny;
  G.nz = h.nz;
  G.bins = ws.bins + 2 * (int64_t)h.bin_half;
  G.hits = ws.sorted + h.hit_base;
  return G;
}

__device__ __forceinline__ void store_state(const Trk& t, int64_t o, const TrackletOut& out) {
  out.x_ref[o] = t.x;
  float* p = out.param + 5 * o;
  p[0] = t.y; p[1] = t.z; p[2] = t.s; p[3] = t.l; p[4] = t.q;
  float* cv = out.cov + 15 * o;
  cv[0] = t.c00; cv[1] = 0.0f; cv[2] = t.d00; cv[3] = t.c10; cv[4] = 0.0f;
  cv[5] = t.c11; cv[6] = 0.0f; cv[7] = t.d10; cv[8] = 0.0f; cv[9] = t.d11;
  cv[10] = t.c20; cv[11] = 0.0f; cv[12] = t.c21; cv[13] = 0.0f; cv[14] = t.c22;
}

__device__ __forceinline__ int stop_flag(int e) { return e == kStepSinPhi ? 2 : 4; }

// Hit-per-row record of one tracklet ([slot][row stride], row stride a
// multiple of 8): a lane collects the aligned chunk of 8 rows it is in (in
// LDS, one int per row and thread) and stores it whole, two 16-byte stores,
// when it moves on, so every record entry is written once and no cache line is
// written back per single hit.
struct RowChunk {
  int32_t* v;  // entry m of this thread at v[m * blockDim]
  int stride;
  int c;       // chunk index (rows 8c .. 8c+7)
};

__device__ __forceinline__ void chunk_clear(RowChunk& k, int c) {
  k.c = c;
#pragma unroll
  for (int m = 0; m < 8; ++m) k.v[m * k.stride] = -1;
}

__device__ __forceinline__ void chunk_set(const RowChunk& k, int r, int32_t idx) { k.v[(r & 7) * k.stride] = idx; }

__device__ __forceinline__ void chunk_store(const RowChunk& k, int32_t* rec) {
  const int32_t* v = k.v;
  const int S = k.stride;
  int4* q = reinterpret_cast<int4*>(rec + 8 * k.c);
  q[0] = make_int4(v[0], v[S], v[2 * S], v[3 * S]);
  q[1] = make_int4(v[4 * S], v[5 * S], v[6 * S], v[7 * S]);
}

__device__ __forceinline__ void chunk_store_none(int c, int32_t* rec) {
  int4* q = reinterpret_cast<int4*>(rec + 8 * c);
  q[0] = make_int4(-1, -1, -1, -1);
  q[1] = make_int4(-1, -1, -1, -1);
}

// Wave totals of the method-step counts (one atomic per wave and counter).
__device__ __forceinline__ void flush_work(const Work& w, const Workspace& ws, int lane) {
  unsigned long long v[4] = {(unsigned long long)w.n_prop, (unsigned long long)w.n_upd,
                             (unsigned long long)w.n_cand, (unsigned long long)w.n_search};
  for (int k = 0; k < 4; ++k) {
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    if (lane == 0 && v[k]) atomicAdd(&ws.counters[kCtrCounts + k], v[k]);
  }
}

// Work partitions of the persistent tracklet kernel (a range of tracklet
// batches).  With nparts == kXcds the range is cut into kXcds contiguous
// parts and a workgroup starts on
// the part of the die it runs on (workgroups are dispatched round-robin over
// the dies), so the row grids a die's L2 holds belong to fewer sectors; a
// wave whose part is used up continues with the following parts.
struct Parts {
  int64_t lo, hi, len;
  int nparts, home;
};

__device__ __forceinline__ Parts make_parts(int64_t lo, int64_t hi, int nparts) {
  Parts P;
  P.lo = lo;
  P.hi = hi;
  P.nparts = nparts;
  P.len = (hi - lo + nparts - 1) / nparts;
  P.home = (int)(blockIdx.x % (unsigned)nparts);
  return P;
}

// Wave-uniform: take `want` consecutive items (batches) from the current part
// (index k, advanced past used-up parts).  Returns the first item and the
// part's end, or -1 when every part is used up.
__device__ __forceinline__ int64_t take_slots(const Parts& P, int& k, unsigned long long* ctr, int want, int lane,
                                              int64_t& part_end) {
  while (k < P.nparts) {
    const int part = (P.home + k) % P.nparts;
    const int64_t plo = P.lo + (int64_t)part * P.len;
    const int64_t phi = min(P.hi, plo + P.len);
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&ctr[part], (unsigned long long)want);
    base = __shfl(base, 0);
    const int64_t s0 = plo + (int64_t)base;
    if (s0 < phi) {
      part_end = phi;
      return s0;
    }
    ++k;
  }
  return -1;
}

constexpr int kTcMaxBlock = 256;

// Bytes of the pad-row planes at the start of the tracklet kernels' dynamic
// LDS (padded to 16 so that what follows stays 16-byte aligned).
__host__ __device__ constexpr int tc_planes_bytes(int R) { return (R * 4 + 15) & ~15; }

// Smallest / largest v over the wave's active lanes, 0 <= v < 2^16, from
// ballots (the result is wave-uniform).
__device__ __forceinline__ int wave_min16(int v) {
  int m = 0;
#pragma unroll
  for (int b = 15; b >= 0; --b)
    if (!__ballot(v < m + (1 << b))) m += 1 << b;
  return m;
}

__device__ __forceinline__ int wave_max16(int v) {
  int m = 0;
#pragma unroll
  for (int b = 15; b >= 0; --b)
    if (__ballot(v >= m + (1 << b))) m += 1 << b;
  return m;
}

// LDS copy of one pad row's grid for a wave's searches (row-synchronous
// form): the header's bin origins, the bin table and the row's sorted hits,
// copied straight from global memory into LDS (global_load_lds, no
// registers; the workgroup size is a multiple of 64, so every wave is whole)
// before the transport arithmetic, so the search that follows the transport
// reads LDS instead of waiting on two dependent global reads.  A row larger
// than kStageBytes is searched in place.
constexpr int kStageBytes = 7168;  // per wave: rows of up to about 290 hits

struct StageLayout {
  int off;   // ints between the 16-byte boundary and the row's first bin (0 or 2)
  int bch;   // 16-byte chunks of bin table
  int bytes; // header's first 16 bytes, bins, hits
};

// The staged copy of a row: [0, 16) the header's first half (bin origins and
// bins per cm), then the bin table from the 16-byte boundary at or below it,
// then the row's hits.
__device__ __forceinline__ StageLayout stage_layout(int ny, int nz, int bin_half, int n) {
  StageLayout L;
  L.off = (2 * bin_half) & 3;
  L.bch = (L.off + ny * nz + 1 + 3) >> 2;
  L.bytes = 16 + 16 * L.bch + 16 * n;
  return L;
}

// Second half of a row header as read ahead: (ny | nz << 16, hit_base,
// bin_half, n).
__device__ __forceinline__ int4 hdr_tail(const Workspace& ws, int64_t i) {
  return reinterpret_cast<const int4*>(ws.hdr + i)[1];
}

// Issue the copies of row i into `reg` (wave-uniform; every lane of the wave
// active: lane j of a copy instruction writes LDS bytes [16 j, 16 j + 16) of
// its destination).  Reads stay inside the header, inside the bin table's
// allocation (the 16-byte chunk holding its last int ends at most 12 bytes
// past it, inside the table's padding) and inside the row's hits.
__device__ __forceinline__ void stage_row(int64_t i, int hit_base, int bin_half, int n, const StageLayout& L,
                                          const Workspace& ws, unsigned char* reg, int lane) {
  // 16-byte chunk c of the copy: 0 the header's first half, 1 .. bch the bin
  // table, then the hits
  const uintptr_t hdr = reinterpret_cast<uintptr_t>(ws.hdr + i);
  const uintptr_t bins = reinterpret_cast<uintptr_t>(ws.bins + (2 * (int64_t)bin_half - L.off));
  const uintptr_t hits = reinterpret_cast<uintptr_t>(ws.sorted + hit_base);
  const int total = 1 + L.bch + n;
  for (int q = 0; q < total; q += 64) {
    const int c = q + lane;
    if (c < total) {
      const uintptr_t src = c == 0 ? hdr : c <= L.bch ? bins + 16 * (uintptr_t)(c - 1) : hits + 16 * (uintptr_t)(c - 1 - L.bch);
      __builtin_amdgcn_global_load_lds((GlobalPtr)src, (LdsPtr)(reg + 16 * q), 16, 0, 0);
    }
  }
}


// Staging state of a wave (row-synchronous form): the staged row's bin counts
// and layout, and the second half of the header of the row the wave steps to
// next, read one row step ahead so that the copies of a row are issued
// without waiting for its header.
struct RowStage {
  int ny, nz;
  StageLayout L;
  int4 pre;
  int pre_s, pre_r;  // sector and row of `pre` (pre_s -1: none)
};

__device__ __forceinline__ RowGrid staged_row_grid(const RowStage& S, unsigned char* reg) {
  const float4 f = *reinterpret_cast<const float4*>(reg);
  RowGrid G;
  G.ymin = f.x; G.zmin = f.y; G.iby = f.z; G.ibz = f.w;
  G.ny = S.ny;
  G.nz = S.nz;
  G.bins = reinterpret_cast<const int32_t*>(reg + 16) + S.L.off;
  G.hits = reinterpret_cast<const SortedHit*>(reg + 16 + 16 * S.L.bch);
  return G;
}

// At the top of a row step, every lane of the wave active: stage row r of the
// wave's sector s (wave-uniform: a batch holds slots of one sector) when a
// lane searches there (`want`) and the copy fits, and read ahead the header of
// row rnext.  Returns whether this lane's search uses the copy.
__device__ __forceinline__ bool stage_for(bool want, int s, int r, int rnext, int R, const Workspace& ws,
                                          unsigned char* reg, int lane, RowStage& S) {
  const unsigned long long m = __ballot(want);
  const int su = __builtin_amdgcn_readfirstlane(s);
  const int ru = __builtin_amdgcn_readfirstlane(r);
  bool mine = false;
  if (m) {
    const int64_t i = (int64_t)su * R + ru;
    const int4 t = (su == S.pre_s && ru == S.pre_r) ? S.pre : hdr_tail(ws, i);
    const int nyz = __builtin_amdgcn_readfirstlane(t.x);
    S.ny = (int16_t)(nyz & 0xffff);
    S.nz = (int16_t)(nyz >> 16);
    if (S.ny > 0) {
      const int hit_base = __builtin_amdgcn_readfirstlane(t.y);
      const int bin_half = __builtin_amdgcn_readfirstlane(t.z);
      const int n = __builtin_amdgcn_readfirstlane(t.w);
      S.L = stage_layout(S.ny, S.nz, bin_half, n);
      if (S.L.bytes <= kStageBytes) {
        stage_row(i, hit_base, bin_half, n, S.L, ws, reg, lane);
        mine = want;
      }
    }
  }
  const int rn = __builtin_amdgcn_readfirstlane(rnext);
  S.pre_s = -1;
  if (rn >= 0 && rn < R) {
    S.pre = hdr_tail(ws, (int64_t)su * R + rn);
    S.pre_s = su;
    S.pre_r = rn;
  }
  return mine;
}

// Profiling build only (-DCATPC_PHASE_CLOCKS=1): shader-clock cycles of the
// row-synchronous tracklet kernel's phases, summed over waves by lane 0 at
// points every lane of the wave reaches (see kPhaseSlots for the layout).  In
// the product build phase_clock() is the constant 0 and nothing is recorded.
#ifndef CATPC_PHASE_CLOCKS
#define CATPC_PHASE_CLOCKS 0
#endif
constexpr bool kPhaseClocks = CATPC_PHASE_CLOCKS != 0;
__device__ unsigned long long g_phase_clocks[kPhaseSlots];

__device__ __forceinline__ unsigned long long phase_clock() {
  if constexpr (kPhaseClocks) return (unsigned long long)clock64();
  return 0ull;
}

// One tracklet: slot -> start hit -> seed chain -> following -> output.
// Every lane of the wave calls it (`valid`: the lane has a slot; `sector`:
// the sector of the wave's batch).  kSync: the
// lanes of a wave walk the pad rows together (a lane whose pass starts later
// waits, a lane whose pass has ended idles), and the row the searching lanes
// need is staged in LDS (`stage`, kStageBytes, this wave's);
// each lane's own sequence of filter steps is the same either way.
template <bool kSync>
__device__ __forceinline__ void build_tracklet(const Inputs& in, int R, const float* __restrict__ row_x, const Consts& c,
                                               const Workspace& ws, int sector, int64_t slot, int64_t o,
                                               bool valid, const TrackletOut& out, int RS, int32_t* chunk_lds,
                                               unsigned char* stage, Work& w) {
  const int lane = threadIdx.x & 63;
  const unsigned long long t_start = phase_clock();
  unsigned n_out = 0, n_in = 0;  // row steps of the two passes (profiling build)
  const int s = sector;
  const int64_t a = in.hit_offset[s];
  int r0 = 0;
  int64_t gi = a;
  if (valid) {
    gi = ws.start_glob[slot];
    r0 = in.row[gi];
  }
  const int32_t h0 = (int32_t)(gi - a);
  int32_t* rec = out.row_hit + o * RS;
  // A start hit has an unlinked hit row below it and two linked rows above
  // it, so on valid input it lies in rows 1 .. R-3.  Only a row value outside
  // the sector's rows fails this (the row check has reported the input as
  // invalid); such a tracklet records nothing and writes nothing outside its
  // own slot.
  const bool in_range = valid && r0 >= 1 && r0 <= R - 3;
  if (valid && !in_range) {
    for (int q = 0; q < RS / 8; ++q) chunk_store_none(q, rec);
    const Trk none = {};
    store_state(none, o, out);
    out.start_row[o] = -1;
    out.first_row[o] = -1;
    out.last_row[o] = -1;
    out.n_hits[o] = 0;
    out.flags[o] = 0;
  }
  ChainHit c0 = {0.0f, 0.0f, -1, 0}, nx = c0, nn = c0;
  if (in_range) {
    c0 = ws.chain[gi];
    nx = ws.chain[a + c0.up];  // next chain measurement
    // the one after it, read one row step ahead so that the pointer chase
    // along the chain overlaps a step of filter arithmetic (a start hit
    // always has an up-link of its up-link)
    nn = nx;
    if (nx.up >= 0) nn = ws.chain[a + nx.up];
  }
  const int k0 = r0 >> 3;  // chunk of the start row
  RowChunk k = {chunk_lds + threadIdx.x, (int)blockDim.x, k0};
  int k_lo = k0, k_hi = k0;  // chunks written
  int fl = 0;
  int nh = 1, first_row = r0, lastr = r0;
  Trk st = {}, snap = {};  // running state; snap: the state the output takes
  bool ok_init = false;
  if (in_range) {
    chunk_clear(k, k0);
    chunk_set(k, r0, h0);
    const int ei = init_track(st, row_x[r0], c0.y, c0.z, row_x[r0 + 1], nx.y, nx.z, c);
    snap = st;  // outward: the state at the last update
    if (ei != kStepOk)
      fl |= stop_flag(ei);
    else
      ok_init = true;
  }
  RowStage S;
  S.pre_s = -1;
  // seed chain (no gate), then outward following
  bool live = ok_init;
  int32_t h = c0.up;
  int miss = 0;
  const int r_first = kSync ? wave_min16(live ? r0 + 1 : R) : r0 + 1;
  const unsigned long long t_out = phase_clock();
  bool fetch = false;  // the chain record after nx is to be read
  for (int r = r_first; r < R; ++r) {
    if (kPhaseClocks) ++n_out;
    bool staged = false;
    if (kSync) {
      if (!__ballot(live)) break;  // every lane's pass has ended
      staged = stage_for(live && r > r0 && h < 0, s, r, r + 1, R, ws, stage, lane, S);
    } else if (!live) {
      break;
    }
    // read at the top of the step, after what the staging waits for: a read
    // issued at the end of the previous step would be waited for here
    if (fetch) {
      nn = ws.chain[a + nx.up];
      fetch = false;
    }
    if (!live || (kSync && r <= r0)) continue;  // ended, or waits for the wave's row
    RowHdr hd;
    if (!kSync && h < 0) hd = ws.hdr[(int64_t)s * R + r];  // issued before the transport arithmetic
    ++w.n_prop;
    const int e = propagate(st, row_x[r], c);
    if (e) {
      fl |= stop_flag(e);
      live = false;
      continue;
    }
    if ((r >> 3) != k.c) {
      chunk_store(k, rec);
      chunk_clear(k, r >> 3);
      k_hi = r >> 3;
    }
    Pick j;
    if (h >= 0) {
      j.idx = h; j.y = nx.y; j.z = nx.z;
    } else if (staged) {
      stage_wait();
      j = closest(st, staged_row_grid(S, stage), c, w);
    } else {
      if (kSync) hd = ws.hdr[(int64_t)s * R + r];
      j = closest(st, grid_of(hd, ws), c, w);
    }
    if (j.idx >= 0) {
      ++w.n_upd;
      if (update(st, j.y, j.z, c)) {
        fl |= 2;
        live = false;
        continue;
      }
      snap = st;
      lastr = r;
      chunk_set(k, r, j.idx);
      ++nh;
      miss = 0;
      if (h >= 0) {
        h = nx.up;
        if (h >= 0) {
          nx = nn;
          fetch = nx.up >= 0;
        }
      }
    } else if (++miss > c.max_miss) {
      live = false;
    }
  }
  const unsigned long long t_back = phase_clock();
  if (in_range) chunk_store(k, rec);
  // back to the start row without updates, then inward following; hits in
  // the start row's chunk (already stored) are written singly, chunks below
  // it are collected as outward
  live = false;
  if (ok_init) {
    st = snap;  // inward: snap becomes the state at the innermost update
    miss = 0;
    k.c = k0;
    live = true;
    for (int r = lastr - 1; r >= r0; --r) {  // back to the start row, no updates
      ++w.n_prop;
      const int e = propagate(st, row_x[r], c);
      if (e) {
        fl |= stop_flag(e);
        live = false;
        break;
      }
    }
    if (live) snap = st;
  }
  const int r_top = (kSync ? wave_max16(live ? r0 : 0) : r0) - 1;
  const unsigned long long t_in = phase_clock();
  for (int r = r_top; r >= 0; --r) {
    if (kPhaseClocks) ++n_in;
    bool staged = false;
    if (kSync) {
      if (!__ballot(live)) break;  // every lane's pass has ended
      staged = stage_for(live && r < r0, s, r, r - 1, R, ws, stage, lane, S);
    } else if (!live) {
      break;
    }
    if (!live || (kSync && r >= r0)) continue;  // ended, or waits for the wave's row
    RowHdr hd;
    if (!kSync) hd = ws.hdr[(int64_t)s * R + r];  // issued before the transport arithmetic
    ++w.n_prop;
    const int e = propagate(st, row_x[r], c);
    if (e) {
      fl |= stop_flag(e);
      live = false;
      continue;
    }
    if ((r >> 3) != k.c) {
      if (k.c < k0) chunk_store(k, rec);
      chunk_clear(k, r >> 3);
      k_lo = r >> 3;
    }
    Pick j;
    if (staged) {
      stage_wait();
      j = closest(st, staged_row_grid(S, stage), c, w);
    } else {
      if (kSync) hd = ws.hdr[(int64_t)s * R + r];
      j = closest(st, grid_of(hd, ws), c, w);
    }
    if (j.idx >= 0) {
      ++w.n_upd;
      if (update(st, j.y, j.z, c)) {
        fl |= 2;
        live = false;
        continue;
      }
      snap = st;
      if (k.c == k0)
        rec[r] = j.idx;
      else
        chunk_set(k, r, j.idx);
      ++nh;
      first_row = r;
      miss = 0;
    } else if (++miss > c.max_miss) {
      live = false;
    }
  }
  if constexpr (kPhaseClocks && kSync) {
    if (lane == 0) {
      const unsigned long long t_end = phase_clock();
      atomicAdd(&g_phase_clocks[kPhaseStart], t_out - t_start);
      atomicAdd(&g_phase_clocks[kPhaseOut], t_back - t_out);
      atomicAdd(&g_phase_clocks[kPhaseBack], t_in - t_back);
      atomicAdd(&g_phase_clocks[kPhaseIn], t_end - t_in);
      atomicAdd(&g_phase_clocks[kPhaseOutSteps], (unsigned long long)n_out);
      atomicAdd(&g_phase_clocks[kPhaseInSteps], (unsigned long long)n_in);
      atomicAdd(&g_phase_clocks[kPhaseBatches], 1ull);
    }
  }
  if (!in_range) return;
  if (ok_init && k.c < k0) chunk_store(k, rec);
  // chunks the passes did not reach
  for (int q = 0; q < k_lo; ++q) chunk_store_none(q, rec);
  for (int q = k_hi + 1; q < RS / 8; ++q) chunk_store_none(q, rec);
  store_state(snap, o, out);
  if (nh >= c.min_hits) fl |= 1;
  if (!spd_ok(snap)) fl |= 8;
  out.start_row[o] = r0;
  out.first_row[o] = first_row;
  out.last_row[o] = lastr;
  out.n_hits[o] = nh;
  out.flags[o] = fl;
}

// Tracklet batches: 64 consecutive slots of one sector (a sector's last batch
// may hold fewer), so that a wave's lanes always search the rows of one
// sector and the row copy serves every one of them.  batch_off[i] = first
// batch of sector s0 + i, i in [0, S]: the exclusive prefix sum of
// ceil(tracklets / 64) over the span's sectors (one workgroup of 1024).
__global__ __launch_bounds__(1024) void k_batches(const int64_t* __restrict__ toff, int s0, int s1,
                                                  int32_t* __restrict__ batch_off) {
  __shared__ int wsum[16];
  const int S = s1 - s0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int carry = 0;
  for (int base = 0; base < S; base += 1024) {
    const int i = base + (int)threadIdx.x;
    const int v = i < S ? (int)((toff[s0 + i + 1] - toff[s0 + i] + 63) >> 6) : 0;
    int incl = v;
    for (int d = 1; d < 64; d <<= 1) {
      const int u = __shfl_up(incl, d);
      if (lane >= d) incl += u;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int before = carry;
    for (int q = 0; q < wv; ++q) before += wsum[q];
    if (i < S) batch_off[i] = before + incl - v;
    int total = 0;
    for (int q = 0; q < 16; ++q) total += wsum[q];
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) batch_off[S] = carry;
}

// Largest i in [0, n) with off[i] <= v (off non-decreasing, off[0] <= v);
// wave-uniform v, so every lane reads the same entries.
template <class T>
__device__ __forceinline__ int last_le(const T* off, int n, int64_t v) {
  int a = 0, b = n;  // off[a] <= v, and off[b] > v or b == n
  while (b - a > 1) {
    const int m = (a + b) >> 1;
    if ((int64_t)off[m] <= v) a = m; else b = m;
  }
  return a;
}

// kWaves > 0 asks the compiler to fit the kernel's registers for at least
// kWaves resident waves per SIMD (spilling to scratch where needed).
// Dynamic LDS: the pad-row planes (R floats, padded to 16 bytes), then, for
// the row-synchronous form, kStageBytes per wave of the workgroup.
template <int kWaves, bool kSync>
__global__ __launch_bounds__(kTcMaxBlock) __attribute__((amdgpu_waves_per_eu(kWaves > 0 ? kWaves : 1))) void
k_tracklets(Inputs in, Span sp, int R, const float* __restrict__ row_x, Consts c, Workspace ws, const int64_t* toff,
            int64_t first, int64_t cap, TrackletOut out, int nparts) {
  __shared__ int32_t chunk_lds[8 * kTcMaxBlock];
  // the pad-row planes in LDS: LDS reads do not wait behind the lane's
  // outstanding memory loads as global reads would
  extern __shared__ __align__(16) unsigned char tc_dyn[];
  float* rxs = reinterpret_cast<float*>(tc_dyn);
  unsigned char* stage = tc_dyn + tc_planes_bytes(R) + (threadIdx.x >> 6) * kStageBytes;
  for (int i = threadIdx.x; i < R; i += blockDim.x) rxs[i] = row_x[i];
  __syncthreads();
  // slots [lo, hi) are tracked; the work queue hands out the batches that
  // cover them
  const int64_t lo = max(toff[sp.s0], first);
  const int64_t hi = min(toff[sp.s1], first + cap);
  const int S = sp.s1 - sp.s0;
  const int lane = threadIdx.x & 63;
  Work w = {0, 0, 0, 0};
  int64_t blo = 0, bhi = 0;
  if (lo < hi) {
    const int i0 = last_le(toff + sp.s0, S, lo), i1 = last_le(toff + sp.s0, S, hi - 1);
    blo = ws.batch_off[i0] + (lo - toff[sp.s0 + i0]) / 64;
    bhi = ws.batch_off[i1] + (hi - 1 - toff[sp.s0 + i1]) / 64 + 1;
  }
  const Parts P = make_parts(blo, bhi, nparts);
  int k = 0;
  const unsigned long long t_wave = phase_clock();
  while (true) {
    int64_t pend = 0;
    const int64_t b = take_slots(P, k, ws.counters + kCtrWork, 1, lane, pend);
    if (b < 0) break;
    const int i = last_le(ws.batch_off, S, b);
    const int64_t slot0 = toff[sp.s0 + i] + 64 * (b - ws.batch_off[i]);
    const int64_t send = min(toff[sp.s0 + i + 1], slot0 + 64);
    const int64_t slot = slot0 + lane;
    build_tracklet<kSync>(in, R, rxs, c, ws, sp.s0 + i, slot, slot - first, slot < send && slot >= lo && slot < hi,
                          out, row_stride(R), chunk_lds, stage, w);
  }
  if constexpr (kPhaseClocks && kSync) {
    if (lane == 0) {
      atomicAdd(&g_phase_clocks[kPhaseWave], phase_clock() - t_wave);
      atomicAdd(&g_phase_clocks[kPhaseWaves], 1ull);
    }
  }
  flush_work(w, ws, lane);
}

// ------------------------------------------------------- tracklet selection
// Of several tracklets that share hits the best keeps them (Sec. 2 item 2):
// the weight of a tracklet is its hit count, then the smaller sector-local
// tracklet index; every hit goes to the heaviest valid tracklet listing it
// (one 64-bit atomic maximum per hit, so the result does not depend on the
// order of the atomics); a tracklet is selected when it keeps at least
// min_hits hits, and its track is the list of hits it keeps, rows ascending.
// 32-bit weight: the hit count (at most R, in hbits = bits of R) above the
// complement of the tracklet index (the remaining bits; a sector with more
// tracklets than they hold is reported, not selected).
__device__ __forceinline__ unsigned sel_weight(int32_t n, int32_t t, int lbits) {
  const unsigned lmask = (1u << lbits) - 1u;
  return ((unsigned)n << lbits) | (lmask - ((unsigned)t & lmask));
}

__host__ __device__ inline int sel_index_bits(int R) {
  int hb = 0;
  while ((1 << hb) <= R) ++hb;
  return 32 - hb;
}

// Slots of the selection: the tracklets present in the output buffer
// (`slots` = its capacity, clamped to the workspace's slot count).
__device__ __forceinline__ int64_t sel_slots(const int64_t* toff, int S, int64_t slots) {
  return max((int64_t)0, min(toff[S], slots));
}


// The emit kernel gives each tracklet 16 lanes (4 tracklets per wave): lane l
// of a group reads the 16-byte pieces l, l+16, l+32 of the record, so the
// record is read with coalesced loads and the per-hit work of a tracklet is
// spread over its lanes.  Persistent grid-stride loop over the slots.
constexpr int kSelLanes = 16;


// Claim: one workgroup per (sector, chunk of kSelRows rows).  The owner
// words of the chunk's hits (contiguous, the hits being sorted by row) are
// kept in LDS while every valid tracklet of the sector takes the atomic
// maximum of its weight on its hits in these rows; then each valid tracklet
// reads back which of its hits in these rows it owns and writes them as the
// chunk's 16-bit kept-row mask.  A chunk with more hits than the LDS holds
// works on the owner words in memory instead.
static_assert(kSelRows == 16, "one 16-bit kept-row mask per chunk");

// Clears the selection's error bits before a selection.
__global__ void k_sel_flags(Workspace ws) {
  if (threadIdx.x == 0) atomicAnd(&ws.counters[kCtrError], ~(2ull | 4ull | 16ull));
}

constexpr int kSelLdsWords = 8192;

__global__ __launch_bounds__(256) void k_sel_claim(Inputs in, int S, const int64_t* toff, int64_t slots, int R,
                                                   TrackletOut trk, Workspace ws) {
  __shared__ unsigned own[kSelLdsWords];
  __shared__ int32_t rfc[kSelRows + 1];  // sector-local first hit of the chunk's rows (and the end)
  const int nch = sel_chunks(R);
  const int s = (int)(blockIdx.x / nch);
  const int r0 = (int)(blockIdx.x % nch) * kSelRows;
  const int r1 = min(R, r0 + kSelRows);
  const int64_t n = sel_slots(toff, S, slots);
  if (blockIdx.x == 0 && threadIdx.x == 0 && toff[S] > slots) atomicOr(&ws.counters[kCtrError], 2ull);
  const int32_t* rf = ws.row_first + (int64_t)s * (R + 1);
  const int32_t h_lo = rf[r0], h_hi = rf[r1];
  const int nh = h_hi - h_lo;
  const int64_t a = in.hit_offset[s];
  unsigned* gown = ws.owner + a + h_lo;
  const bool lds = nh <= kSelLdsWords;
  for (int k = threadIdx.x; k < nh; k += blockDim.x) {
    if (lds) own[k] = 0u; else gown[k] = 0u;
  }
  for (int k = threadIdx.x; k <= r1 - r0; k += blockDim.x) rfc[k] = rf[r0 + k];
  if (!lds) __threadfence();
  __syncthreads();
  const int lbits = sel_index_bits(R);
  const int64_t t0 = min(toff[s], n), t1 = min(toff[s + 1], n);
  const int RS = row_stride(R);
  bool bad = false, many = false;
  // A thread's first tracklet keeps its record piece (these rows) in
  // registers for the second pass; further tracklets read theirs again.
  constexpr int kQ = kSelRows / 4;
  const int nq = (r1 - r0 + 3) / 4;
  int4 keep[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) keep[q] = make_int4(-1, -1, -1, -1);
  for (int64_t slot = t0 + threadIdx.x; slot < t1; slot += blockDim.x) {
    if (!(trk.flags[slot] & 1)) continue;
    const int32_t local = (int32_t)(slot - toff[s]);
    if (local >= (1 << lbits)) { many = true; continue; }
    const unsigned key = sel_weight(trk.n_hits[slot], local, lbits);
    const int4* rec = reinterpret_cast<const int4*>(trk.row_hit + slot * RS + r0);
    int4 vq[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) vq[q] = q < nq ? rec[q] : make_int4(-1, -1, -1, -1);
    if (slot == t0 + threadIdx.x) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) keep[q] = vq[q];
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int4 v = vq[q];
      const int32_t hv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int32_t h = hv[m];
        const int rr = 4 * q + m;
        if (h < 0 || rr >= r1 - r0) continue;
        if (h < rfc[rr] || h >= rfc[rr + 1]) { bad = true; continue; }  // not a hit of the entry's row
        const int32_t hl = h - h_lo;
        if (lds) atomicMax(&own[hl], key); else atomicMax(&gown[hl], key);
      }
    }
  }
  if (bad) atomicOr(&ws.counters[kCtrError], 4ull);
  if (many) atomicOr(&ws.counters[kCtrError], 16ull);
  if (!lds) __threadfence();
  __syncthreads();
  // The owner words are final: the kept rows of each valid tracklet here.
  const int ch = r0 / kSelRows;
  for (int64_t slot = t0 + threadIdx.x; slot < t1; slot += blockDim.x) {
    if (!(trk.flags[slot] & 1)) continue;
    const int32_t local = (int32_t)(slot - toff[s]);
    unsigned bits = 0u;
    if (local < (1 << lbits)) {  // past the index limit a tracklet owns nothing
      const unsigned key = sel_weight(trk.n_hits[slot], local, lbits);
      const int4* rec = reinterpret_cast<const int4*>(trk.row_hit + slot * RS + r0);
      const bool kept = slot == t0 + threadIdx.x;
      int4 vq[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) vq[q] = kept ? keep[q] : q < nq ? rec[q] : make_int4(-1, -1, -1, -1);
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int4 v = vq[q];
        const int32_t hv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int rr = 4 * q + m;
          if (hv[m] < 0 || rr >= r1 - r0) continue;
          if (hv[m] < rfc[rr] || hv[m] >= rfc[rr + 1]) continue;  // reported by the first pass
          const int32_t hl = hv[m] - h_lo;
          // in memory the words were set by atomics at the device level: read them there
          const unsigned o = lds ? own[hl] : __hip_atomic_load(&gown[hl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (o == key) bits |= 1u << (4 * q + m);
        }
      }
    }
    ws.sel_mask[slot * nch + ch] = (uint16_t)bits;
    if (ch == 0) ws.sel_local[slot] = local;  // for the emit pass
  }
}

// Count: one lane per slot, the kept rows of a valid tracklet from its
// per-chunk masks.
__global__ __launch_bounds__(256) void k_sel_count(const int64_t* toff, int S, int64_t slots, int R,
                                                   TrackletOut trk, Consts c, Workspace ws) {
  const int64_t n = sel_slots(toff, S, slots);
  const int nch = sel_chunks(R);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; slot < n; slot += stride) {
    int cnt = -1;
    if (trk.flags[slot] & 1) {
      cnt = 0;
      for (int k = 0; k < nch; ++k) cnt += __popc((unsigned)ws.sel_mask[slot * nch + k]);
      if (cnt < c.min_hits) cnt = -1;
    }
    ws.sel_cnt[slot] = cnt;
  }
}

// Exclusive scans over the slots: selected tracks and their kept hits, 1024
// slots per workgroup (offsets relative to the group), then the group totals.
__global__ __launch_bounds__(kScanGroup) void k_sel_scan_local(const int64_t* toff, int S, int64_t slots,
                                                                 Workspace ws) {
  __shared__ int wsum[2][kScanGroup / 64];
  const int64_t n = sel_slots(toff, S, slots);
  const int64_t b = (int64_t)blockIdx.x * kScanGroup + threadIdx.x;
  const int cv = b < n ? ws.sel_cnt[b] : -1;
  const int vt = cv >= 0 ? 1 : 0, vh = cv >= 0 ? cv : 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int it = vt, ih = vh;
  for (int o = 1; o < 64; o <<= 1) {
    const int ut = __shfl_up(it, o), uh = __shfl_up(ih, o);
    if (lane >= o) { it += ut; ih += uh; }
  }
  if (lane == 63) { wsum[0][wave] = it; wsum[1][wave] = ih; }
  __syncthreads();
  if (wave == 0) {
    int xt = lane < kScanGroup / 64 ? wsum[0][lane] : 0, xh = lane < kScanGroup / 64 ? wsum[1][lane] : 0;
    for (int o = 1; o < kScanGroup / 64; o <<= 1) {
      const int ut = __shfl_up(xt, o), uh = __shfl_up(xh, o);
      if (lane >= o) { xt += ut; xh += uh; }
    }
    if (lane < kScanGroup / 64) { wsum[0][lane] = xt; wsum[1][lane] = xh; }
  }
  __syncthreads();
  if (b <= n) {
    const int bt = wave ? wsum[0][wave - 1] : 0, bh = wave ? wsum[1][wave - 1] : 0;
    ws.sel_loc[b] = make_int2(bt + it - vt, bh + ih - vh);
  }
  if (threadIdx.x == kScanGroup - 1)
    ws.sel_grp[blockIdx.x] = make_longlong2(wsum[0][kScanGroup / 64 - 1], wsum[1][kScanGroup / 64 - 1]);
}

__global__ __launch_bounds__(1024) void k_sel_scan_top(int64_t ng, Workspace ws) {
  __shared__ int64_t pt[1024], ph[1024];
  const int t = threadIdx.x;
  const int64_t per = (ng + 1023) / 1024;
  const int64_t g0 = min(ng, (int64_t)t * per), g1 = min(ng, g0 + per);
  int64_t st = 0, sh = 0;
  for (int64_t g = g0; g < g1; ++g) { st += ws.sel_grp[g].x; sh += ws.sel_grp[g].y; }
  pt[t] = st;
  ph[t] = sh;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t vt = t >= o ? pt[t - o] : 0, vh = t >= o ? ph[t - o] : 0;
    __syncthreads();
    pt[t] += vt;
    ph[t] += vh;
    __syncthreads();
  }
  int64_t rt = pt[t] - st, rh = ph[t] - sh;
  for (int64_t g = g0; g < g1; ++g) {
    const longlong2 v = ws.sel_grp[g];
    ws.sel_grp[g] = make_longlong2(rt, rh);
    rt += v.x;
    rh += v.y;
  }
  if (t == 1023) {
    ws.sel_grp[ng] = make_longlong2(pt[1023], ph[1023]);
    ws.counters[kCtrSelTracks] = (unsigned long long)pt[1023];
    ws.counters[kCtrSelHits] = (unsigned long long)ph[1023];
  }
}

__device__ __forceinline__ longlong2 sel_offset(const Workspace& ws, int64_t b) {
  const longlong2 g = ws.sel_grp[b / kScanGroup];
  const int2 l = ws.sel_loc[b];
  return make_longlong2(g.x + l.x, g.y + l.y);
}

// Each selected tracklet writes its track (16 lanes, the kept hits in row
// order through a prefix count over the lanes); the grid's first S+1 threads
// also write the first track of each sector.
__global__ __launch_bounds__(256) void k_sel_emit(Inputs in, int S, const int64_t* toff, int64_t slots, int R,
                                                  TrackletOut trk, Workspace ws, TracksOut out) {
  const int64_t n = sel_slots(toff, S, slots);
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = gtid; s <= S; s += nthreads) {
    const int64_t q = max((int64_t)0, min(toff[s], n));
    out.track_offset[s] = sel_offset(ws, q).x;
  }
  const int sub = threadIdx.x & (kSelLanes - 1);
  const int64_t stride = nthreads / kSelLanes;
  const int RS4 = row_stride(R) / 4;
  const int nch = sel_chunks(R);
  for (int64_t slot = gtid / kSelLanes; slot < n; slot += stride) {
    const int cnt = ws.sel_cnt[slot];
    if (cnt < 0) continue;  // the 16 lanes of a slot take this branch together
    const longlong2 off = sel_offset(ws, slot);
    if (sub == 0 && off.x < out.track_capacity) {
      out.track_tracklet[off.x] = ws.sel_local[slot];
      out.track_n_hits[off.x] = cnt;
      out.track_hit_offset[off.x] = off.y;
    }
    const int4* rec = reinterpret_cast<const int4*>(trk.row_hit + slot * row_stride(R));
    int64_t base = off.y;
    for (int q0 = 0; q0 < RS4; q0 += kSelLanes) {
      const int q = q0 + sub;
      int32_t w[4] = {-1, -1, -1, -1};
      bool own[4] = {false, false, false, false};
      int mine = 0;
      if (q < RS4) {
        const int4 v = rec[q];
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        // rows 4q..4q+3 of the claim's kept-row mask (chunk q / 4; 4q < row_stride(R) <= 16 * nch)
        const unsigned bits = (unsigned)ws.sel_mask[slot * nch + (q >> 2)] >> (4 * (q & 3));
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          own[m] = ((bits >> m) & 1u) != 0u;
          mine += own[m];
        }
      }
      // kept hits of the lanes before this one in this round (rows ascend with q)
      int incl = mine;
      for (int o = 1; o < kSelLanes; o <<= 1) {
        const int u = __shfl_up(incl, o, kSelLanes);
        if (sub >= o) incl += u;
      }
      int64_t k = base + incl - mine;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (!own[m]) continue;
        if (k < out.hit_capacity) out.track_hits[k] = w[m];
        ++k;
      }
      base += __shfl(incl, kSelLanes - 1, kSelLanes);
    }
  }
}

// ------------------------------------------------------ full Kalman refit
// Sec. 2 item 4: the final fit with the full Kalman filter, here of each
// selected track: full 5x5 covariance over (y, z, sin phi, tan lambda, q/pT),
// the tracklet filter's helix transport of the state, covariance C <- F C F^T
// with the first-order Jacobian including the terms that couple z to
// (sin phi, q/pT), 2-d updates with (y, z); start from the tracklet's
// parameters carried to the innermost hit, prior diag(sy^2, sz^2, 1, 1, 100);
// result at the outermost hit.  One lane per track, in binary64 (MI355X runs
// binary64 vector arithmetic at the binary32 rate; in binary32 the long
// coupled covariance products lose about 1e-3 cm in z and 1e-3 in q/pT).
// The matrix products run, in a fixed order, over the entries of F that are
// not zero by construction.
__device__ __forceinline__ int ff_tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

struct FitJac {
  double a, b, d, e, f, dS;  // dy/ds, dy/dq, ds/dq, dz/ds, dz/dq, dz/dl
};

__device__ __forceinline__ double ff_F(const FitJac& J, int i, int j) {
  if (i == j) return 1.0;
  if (i == 0 && j == 2) return J.a;
  if (i == 0 && j == 4) return J.b;
  if (i == 1 && j == 2) return J.e;
  if (i == 1 && j == 3) return J.dS;
  if (i == 1 && j == 4) return J.f;
  if (i == 2 && j == 4) return J.d;
  return 0.0;
}

// Structurally nonzero entries of F (the identity and a, b, e, dS, f, d):
// the covariance products skip the others.  A skipped term would add +-0 to
// a running sum that starts at +0, which leaves it unchanged for finite
// covariances, so the order and rounding of the remaining terms are those of
// the full sum.
__host__ __device__ constexpr bool ff_nz(int i, int j) {
  return i == j || (i == 0 && (j == 2 || j == 4)) || (i == 1 && j >= 2) || (i == 2 && j == 4);
}

// State transport to x1 (the tracklet filter's formulas) and the Jacobian.
__device__ __forceinline__ int ff_transport(double& x, double* p, double x1, double kb, FitJac* J) {
  const double dx = x1 - x;
  const double k = kb * p[4];
  const double s0 = p[2];
  const double s1 = s0 + k * dx;
  if (!(fabs(s1) < 0.999)) return 2;
  const double c0 = sqrt(1.0 - s0 * s0);
  const double c1 = sqrt(1.0 - s1 * s1);
  const double T = (s0 + s1) / (c0 + c1);
  const double dy = dx * T;
  const double ch = sqrt(dx * dx + dy * dy);
  const double u = (k * ch) * 0.5;
  if (!(fabs(u) <= 0.2)) return 4;
  const double u2 = u * u;
  const double A = 1.0 + u2 * (1.0 / 6.0 + u2 * (3.0 / 40.0 + u2 * (5.0 / 112.0 + u2 * (35.0 / 1152.0))));
  double dS = ch * A;
  if (dx < 0.0) dS = -dS;
  if (J) {
    const double sm = (s0 + s1) * 0.5;
    const double cm2 = 1.0 - sm * sm;
    const double cm3 = cm2 * sqrt(cm2);
    J->a = dx / cm3;
    J->b = ((kb * dx) * dx * 0.5) / cm3;
    J->d = kb * dx;
    J->e = ((p[3] * dx) * sm) / cm3;
    J->f = (J->e * J->d) * 0.5;
    J->dS = dS;
  }
  x = x1;
  p[0] = p[0] + dy;
  p[1] = p[1] + p[3] * dS;
  p[2] = s1;
  return 0;
}

__device__ __forceinline__ void ff_transport_cov(double* C, const FitJac& J) {
  double M[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 5; ++k)
        if (ff_nz(i, k)) acc = acc + ff_F(J, i, k) * C[ff_tri(k, j)];
      M[i][j] = acc;
    }
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 5; ++k)
        if (ff_nz(j, k)) acc = acc + M[i][k] * ff_F(J, j, k);
      C[ff_tri(i, j)] = acc;
    }
}

__device__ __forceinline__ int ff_update(double* p, double* C, double my, double mz, double sy2, double sz2,
                                         double& chi2) {
  const double r0 = my - p[0];
  const double r1 = mz - p[1];
  const double S00 = C[ff_tri(0, 0)] + sy2;
  const double S01 = C[ff_tri(1, 0)];
  const double S11 = C[ff_tri(1, 1)] + sz2;
  const double det = S00 * S11 - S01 * S01;
  if (!(det > 0.0)) return 8;
  const double i00 = S11 / det;
  const double i01 = (0.0 - S01) / det;
  const double i11 = S00 / det;
  double K[5][2];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    K[i][0] = C[ff_tri(i, 0)] * i00 + C[ff_tri(i, 1)] * i01;
    K[i][1] = C[ff_tri(i, 0)] * i01 + C[ff_tri(i, 1)] * i11;
  }
  const double s_new = p[2] + (K[2][0] * r0 + K[2][1] * r1);
  if (!(fabs(s_new) < 0.999)) return 2;
#pragma unroll
  for (int i = 0; i < 5; ++i) p[i] = p[i] + (K[i][0] * r0 + K[i][1] * r1);
  double Cn[15];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      Cn[ff_tri(i, j)] = C[ff_tri(i, j)] - (K[i][0] * C[ff_tri(0, j)] + K[i][1] * C[ff_tri(1, j)]);
#pragma unroll
  for (int q = 0; q < 15; ++q) C[q] = Cn[q];
  chi2 = chi2 + (r0 * (i00 * r0 + i01 * r1) + r1 * (i01 * r0 + i11 * r1));
  return 0;
}

__global__ __launch_bounds__(256) void k_fullfit(Inputs in, int S, int R, const float* __restrict__ row_x,
                                                 Consts c, const int64_t* toff, TrackletOut trk, int64_t trk_cap,
                                                 TracksOut tr, FitsOut out, Workspace ws) {
  // the row positions in LDS (R floats of dynamic LDS): read at every row step
  extern __shared__ __align__(16) unsigned char ff_dyn[];
  float* rxs = reinterpret_cast<float*>(ff_dyn);
  for (int r = threadIdx.x; r < R; r += blockDim.x) rxs[r] = row_x[r];
  __syncthreads();
  const int64_t n = min(tr.track_offset[S], min(tr.track_capacity, out.capacity));
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
    const int s = sector_of(tr.track_offset, 0, S, t);
    const int64_t a = in.hit_offset[s];
    const int32_t ns = (int32_t)(in.hit_offset[s + 1] - a);
    const int64_t slot = toff[s] + tr.track_tracklet[t];
    const int nh = tr.track_n_hits[t];
    const int64_t h0 = tr.track_hit_offset[t];
    double x = 0.0, p[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, C[15];
#pragma unroll
    for (int q = 0; q < 15; ++q) C[q] = 0.0;
    double chi2 = 0.0;
    int fl = 0, used = 0;
    bool ok = nh > 0 && slot >= 0 && slot < trk_cap && h0 >= 0 && h0 + nh <= tr.hit_capacity;
    int32_t h_first = 0, h_last = 0;
    if (ok) {
      h_first = tr.track_hits[h0];
      h_last = tr.track_hits[h0 + nh - 1];
      ok = h_first >= 0 && h_first < ns && h_last >= 0 && h_last < ns;
    }
    const int start_row = ok ? trk.first_row[slot] : 0;
    const int r_first = ok ? in.row[a + h_first] : 0, r_last = ok ? in.row[a + h_last] : 0;
    if (!ok || r_first < start_row || r_last >= R || start_row < 0) {
      fl = 64;
    } else {
      x = (double)trk.x_ref[slot];
#pragma unroll
      for (int i = 0; i < 5; ++i) p[i] = (double)trk.param[5 * slot + i];
      // The hit data are read ahead: when hit k is used, the row, y and z of
      // hit k+1 and the index of hit k+2 are already on their way.
      const float* yv = in.y + a;
      const float* zv = in.z + a;
      const int32_t* rv = in.row + a;
      const int32_t* hv = tr.track_hits + h0;
      float yk = yv[h_first], zk = zv[h_first];
      int32_t h1 = nh > 1 ? hv[1] : -1, h2 = nh > 2 ? hv[2] : -1;
      int r1 = 0;
      float y1 = 0.f, z1 = 0.f;
      if (h1 >= 0 && h1 < ns) { r1 = rv[h1]; y1 = yv[h1]; z1 = zv[h1]; }
      for (int r = start_row + 1; r <= r_first && !fl; ++r)
        fl = ff_transport(x, p, (double)rxs[r], c.kbd, nullptr);
      if (!fl) {
        C[ff_tri(0, 0)] = c.sy2d;
        C[ff_tri(1, 1)] = c.sz2d;
        C[ff_tri(2, 2)] = 1.0;
        C[ff_tri(3, 3)] = 1.0;
        C[ff_tri(4, 4)] = 100.0;
        int k = 0;
        int rk = r_first;
        for (int r = r_first; r <= r_last; ++r) {
          if (r > r_first) {
            FitJac J;
            fl = ff_transport(x, p, (double)rxs[r], c.kbd, &J);
            if (fl) break;
            ff_transport_cov(C, J);
          }
          if (k < nh && rk == r) {
            fl = ff_update(p, C, (double)yk, (double)zk, c.sy2d, c.sz2d, chi2);
            if (fl) break;
            ++k;
            ++used;
            if (k < nh) {
              if (h1 < 0 || h1 >= ns) { fl = 64; break; }  // hit k
              rk = r1;
              yk = y1;
              zk = z1;
              h1 = h2;  // hit k+1
              if (k + 1 < nh && h1 >= 0 && h1 < ns) { r1 = rv[h1]; y1 = yv[h1]; z1 = zv[h1]; }
              if (k + 2 < nh) h2 = hv[k + 2];
            }
          }
        }
        if (!fl) fl = 1;
      }
    }
    out.x[t] = (float)x;
#pragma unroll
    for (int i = 0; i < 5; ++i) out.param[5 * t + i] = (float)p[i];
#pragma unroll
    for (int q = 0; q < 15; ++q) out.cov[15 * t + q] = (float)C[q];
    out.chi2[t] = (float)chi2;
    out.ndf[t] = 2 * used - 5;
    out.flags[t] = fl;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && tr.track_offset[S] > min(tr.track_capacity, out.capacity))
    atomicOr(&ws.counters[kCtrError], 32ull);
}

// ------------------------------------------------- segment merging
// Per track, for the candidate scan: the tracklet's start x, y, z and its
// first row | (row of the track's outermost hit << 16), or -1 in .w when the
// track takes no part (refit not done, or an inconsistent record).  Also
// resets the outputs, both best-partner keys and the pair counter.
__global__ __launch_bounds__(256) void k_merge_prep(Inputs in, int S, int R, const int64_t* toff, TrackletOut trk,
                                                    int64_t trk_cap, TracksOut tr, FitsOut fits, MergeOut out,
                                                    Workspace ws, int64_t n_max) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ws.counters[kCtrMergePairs] = 0ull;
    ws.counters[kCtrMergeSteps] = 0ull;
  }
  const int64_t n = min(tr.track_offset[S], n_max);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
    const int s = sector_of(tr.track_offset, 0, S, t);
    const int64_t a = in.hit_offset[s];
    const int32_t ns = (int32_t)(in.hit_offset[s + 1] - a);
    const int64_t slot = toff[s] + tr.track_tracklet[t];
    const int nh = tr.track_n_hits[t];
    const int64_t h0 = tr.track_hit_offset[t];
    bool ok = fits.flags[t] == 1 && nh > 0 && slot >= 0 && slot < trk_cap && h0 >= 0 && h0 + nh <= tr.hit_capacity;
    int32_t hl = 0, last = 0, first = 0;
    if (ok) {
      hl = tr.track_hits[h0 + nh - 1];
      ok = hl >= 0 && hl < ns;
    }
    if (ok) {
      last = in.row[a + hl];
      first = trk.first_row[slot];
      ok = last >= 0 && last < R && first >= 0 && first < R;
    }
    float4 rec = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
    if (ok) rec = make_float4(trk.x_ref[slot], trk.param[5 * slot], trk.param[5 * slot + 1], __int_as_float(first | (last << 16)));
    ws.mrec[t] = rec;
    ws.mslot[t] = ok ? (int32_t)slot : -1;
    ws.mkey_a[t] = ~0ull;
    ws.mkey_b[t] = ~0ull;
    ws.mover[t] = 0;
    out.next[t] = -1;
    out.prev[t] = -1;
    out.head[t] = (int32_t)t;
    out.chi2[t] = -1.f;
  }
}

// chi^2 of segment A's end state against the start state of a continuation B
// (A carried row by row with the refit's transport and Jacobian), or -1 when
// the transport stops or the summed covariance is not positive definite.
__device__ __forceinline__ double merge_chi2(int64_t A, int64_t B, const float* __restrict__ row_x, double kb,
                                             const TrackletOut& trk, const FitsOut& fits, const Workspace& ws,
                                             int& steps) {
  const int a_last = __float_as_int(ws.mrec[A].w) >> 16;
  const int b_first = __float_as_int(ws.mrec[B].w) & 0xffff;
  const int64_t sb = ws.mslot[B];
  const float* __restrict__ bp = trk.param + 5 * sb;
  const float* __restrict__ bC = trk.cov + 15 * sb;
  double x = (double)fits.x[A], p[5], C[15];
#pragma unroll
  for (int i = 0; i < 5; ++i) p[i] = (double)fits.param[5 * A + i];
#pragma unroll
  for (int q = 0; q < 15; ++q) C[q] = (double)fits.cov[15 * A + q];
  for (int r = a_last + 1; r <= b_first; ++r) {
    FitJac J;
    if (ff_transport(x, p, (double)row_x[r], kb, &J)) return -1.0;
    ff_transport_cov(C, J);
    ++steps;
  }
  double d[5], L[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i) d[i] = (double)bp[i] - p[i];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) L[i][j] = 0.0;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double acc = C[ff_tri(i, j)] + (double)bC[ff_tri(i, j)];
#pragma unroll
      for (int q = 0; q < j; ++q) acc = acc - L[i][q] * L[j][q];
      if (i == j) {
        if (!(acc > 0.0)) return -1.0;
        L[i][i] = sqrt(acc);
      } else {
        L[i][j] = acc / L[j][j];
      }
    }
  double w[5], chi2 = 0.0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    double acc = d[i];
#pragma unroll
    for (int q = 0; q < i; ++q) acc = acc - L[i][q] * w[q];
    w[i] = acc / L[i][i];
    chi2 = chi2 + w[i] * w[i];
  }
  return chi2;
}

// A compatible pair takes the atomic minimum of (chi^2 bits, partner) on both
// keys: A's key ends at its best continuation, B's at its best predecessor,
// whatever the order of the atomics (chi^2 >= 0, so its bits order as the
// values; equal values order by the index).
__device__ __forceinline__ void merge_pair(int64_t A, int64_t B, const float* __restrict__ row_x, const Consts& c,
                                           const MergeCuts& m, const TrackletOut& trk, const FitsOut& fits,
                                           const Workspace& ws, int& steps) {
  const double chi2 = merge_chi2(A, B, row_x, c.kbd, trk, fits, ws, steps);
  if (!(chi2 >= 0.0 && chi2 <= m.chi2_max)) return;
  const unsigned long long hi = (unsigned long long)__float_as_uint((float)chi2) << 32;
  atomicMin(&ws.mkey_a[A], hi | (unsigned long long)(uint32_t)B);
  atomicMin(&ws.mkey_b[B], hi | (unsigned long long)(uint32_t)A);
}

// The cheap tests of a pair (rows, straight-line window) for segment A
// against every segment B of its sector; f(B) for each pair that passes.
template <class F>
__device__ __forceinline__ void merge_scan(int64_t A, int64_t n, int S, const MergeCuts& m, const TracksOut& tr,
                                           const FitsOut& fits, const Workspace& ws, F&& f) {
  const int wa = __float_as_int(ws.mrec[A].w);
  if (wa < 0) return;
  const int a_last = wa >> 16;
  const int s = sector_of(tr.track_offset, 0, S, A);
  const int64_t k0 = tr.track_offset[s], k1 = min(tr.track_offset[s + 1], n);
  const double ax = (double)fits.x[A];
  const double ay = (double)fits.param[5 * A], az = (double)fits.param[5 * A + 1];
  const double as = (double)fits.param[5 * A + 2], al = (double)fits.param[5 * A + 3];
  const double ca = sqrt(1.0 - as * as);
  const double ty = as / ca, tz = al / ca;
  for (int64_t B = k0; B < k1; ++B) {
    const float4 rb = ws.mrec[B];
    const int wb = __float_as_int(rb.w);
    if (B == A || wb < 0) continue;
    const int b_first = wb & 0xffff;
    if (!(b_first > a_last && b_first - a_last <= m.max_gap)) continue;
    const double dx0 = (double)rb.x - ax;
    const double yw = (ay + dx0 * ty) - (double)rb.y;
    const double zw = (az + dx0 * tz) - (double)rb.z;
    if (!(fabs(yw) <= m.window && fabs(zw) <= m.window)) continue;
    f(B, s);
  }
}

// Chunks of 256 segments per sector and their exclusive prefix over the
// sectors (one workgroup of 1024; sectors in tiles of 1024).
__global__ __launch_bounds__(1024) void k_merge_chunks(int S, TracksOut tr, Workspace ws, int64_t n_max) {
  __shared__ int part[1024];
  const int64_t n = min(tr.track_offset[S], n_max);
  int carry = 0;
  for (int base = 0; base < S; base += 1024) {
    const int s = base + threadIdx.x;
    int v = 0;
    if (s < S) {
      const int64_t k0 = min(tr.track_offset[s], n), k1 = min(tr.track_offset[s + 1], n);
      v = (int)((k1 - k0 + 255) / 256);
    }
    part[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int add = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
      __syncthreads();
      part[threadIdx.x] += add;
      __syncthreads();
    }
    if (s < S) ws.mchunk[s] = carry + part[threadIdx.x] - v;
    carry += part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) ws.mchunk[S] = carry;
}

// One workgroup per chunk of 256 segments of a sector, one lane per segment
// A; the sector's segment records are staged in LDS in tiles and every lane
// walks the same tile entry at the same time (a broadcast read), so the walk
// is uniform across the wave.  A lane queues up to kMergeQueue partners B
// that pass the cheap tests in registers; when a queue is full, and at the
// end of the chunk, the wave writes all queues to the list at positions
// reserved with one atomic (a counter hit once per pair serialises in L2).
// A segment with a pair beyond the list is marked for k_merge_over.
constexpr int kMergeTile = 2048;  // segment records per LDS tile (32 KiB)
constexpr int kMergeQueue = 4;    // partners a lane holds before the wave writes them out

__device__ __forceinline__ void merge_flush(int64_t A, int qn, int32_t q0, int32_t q1, int32_t q2, int32_t q3,
                                            int lane, int64_t pair_cap, Workspace& ws) {
  // qn in [0, 4]: the wave's total and this lane's offset from the bits of qn
  const unsigned long long below = (1ull << lane) - 1ull;
  const unsigned long long b0 = __ballot(qn & 1), b1 = __ballot(qn & 2), b2 = __ballot(qn & 4);
  const int total = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
  if (total == 0) return;
  const int off = __popcll(b0 & below) + 2 * __popcll(b1 & below) + 4 * __popcll(b2 & below);
  unsigned long long g = 0ull;
  if (lane == 0) g = atomicAdd(&ws.counters[kCtrMergePairs], (unsigned long long)total);
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)g, 0);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(g >> 32), 0);
  const int64_t base = (int64_t)(((unsigned long long)hi << 32) | lo) + off;
  // the lane's queued partners are q0 .. q[qn - 1]
  const int32_t q[kMergeQueue] = {q0, q1, q2, q3};
#pragma unroll
  for (int j = 0; j < kMergeQueue; ++j) {
    if (j < qn) {
      const int64_t k = base + j;
      if (k < pair_cap)
        ws.mpair[k] = make_int2((int32_t)A, q[j]);
      else
        ws.mover[A] = 1;
    }
  }
}

__global__ __launch_bounds__(256) void k_merge_cand(int S, MergeCuts m, TracksOut tr, FitsOut fits, Workspace ws,
                                                    int64_t n_max, int64_t pair_cap) {
  __shared__ float4 recs[kMergeTile];
  const int64_t n = min(tr.track_offset[S], n_max);
  const int lane = threadIdx.x & 63;
  const int total = ws.mchunk[S];
  for (int v = blockIdx.x; v < total; v += gridDim.x) {
    // sector of this chunk of 256 segments: largest s with mchunk[s] <= v
    int lo = 0, hi = S;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (ws.mchunk[mid] <= v) lo = mid; else hi = mid;
    }
    const int s = lo;
    const int64_t k0 = min(tr.track_offset[s], n), k1 = min(tr.track_offset[s + 1], n);
    const int64_t A = k0 + (int64_t)(v - ws.mchunk[s]) * 256 + threadIdx.x;
    int a_last = -1;
    double ax = 0.0, ay = 0.0, az = 0.0, ty = 0.0, tz = 0.0;
    if (A < k1) {
      const int wa = __float_as_int(ws.mrec[A].w);
      if (wa >= 0) {
        a_last = wa >> 16;
        ax = (double)fits.x[A];
        ay = (double)fits.param[5 * A];
        az = (double)fits.param[5 * A + 1];
        const double as = (double)fits.param[5 * A + 2], al = (double)fits.param[5 * A + 3];
        const double ca = sqrt(1.0 - as * as);
        ty = as / ca;
        tz = al / ca;
      }
    }
    int qn = 0;
    int32_t q0 = -1, q1 = -1, q2 = -1, q3 = -1;
    for (int64_t b0 = k0; b0 < k1; b0 += kMergeTile) {
      const int nb = (int)min<int64_t>(kMergeTile, k1 - b0);
      __syncthreads();
      for (int i = threadIdx.x; i < nb; i += blockDim.x) recs[i] = ws.mrec[b0 + i];
      __syncthreads();
      for (int i = 0; i < nb; ++i) {
        const float4 rb = recs[i];
        const int wb = __float_as_int(rb.w);
        bool pass = false;
        if (a_last >= 0 && wb >= 0 && b0 + i != A) {
          const int b_first = wb & 0xffff;
          if (b_first > a_last && b_first - a_last <= m.max_gap) {
            const double dx0 = (double)rb.x - ax;
            const double yw = (ay + dx0 * ty) - (double)rb.y;
            const double zw = (az + dx0 * tz) - (double)rb.z;
            pass = fabs(yw) <= m.window && fabs(zw) <= m.window;
          }
        }
        if (pass) {
          q3 = q2;
          q2 = q1;
          q1 = q0;
          q0 = (int32_t)(b0 + i);
          ++qn;
        }
        if (__ballot(qn == kMergeQueue)) {
          merge_flush(A, qn, q0, q1, q2, q3, lane, pair_cap, ws);
          qn = 0;
        }
      }
    }
    merge_flush(A, qn, q0, q1, q2, q3, lane, pair_cap, ws);
  }
}

// Segments marked by k_merge_cand evaluate all their pairs themselves (a
// pair that is also listed gives the same atomic minimum twice).
__global__ __launch_bounds__(256) void k_merge_over(int S, const float* __restrict__ row_x, Consts c, MergeCuts m,
                                                    const int64_t* toff, TrackletOut trk, TracksOut tr, FitsOut fits,
                                                    Workspace ws, int64_t n_max) {
  const int64_t n = min(tr.track_offset[S], n_max);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t A = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; A < n; A += stride) {
    if (!ws.mover[A]) continue;
    int steps = 0;
    merge_scan(A, n, S, m, tr, fits, ws, [&](int64_t B, int) { merge_pair(A, B, row_x, c, m, trk, fits, ws, steps); });
    atomicAdd(&ws.counters[kCtrMergeSteps], (unsigned long long)steps);
  }
}

// One lane per listed pair.
__global__ __launch_bounds__(256) void k_merge_chi2(int S, const float* __restrict__ row_x, Consts c, MergeCuts m,
                                                    const int64_t* toff, TrackletOut trk, TracksOut tr, FitsOut fits,
                                                    Workspace ws, int64_t pair_cap) {
  const int64_t np = min((int64_t)ws.counters[kCtrMergePairs], pair_cap);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int steps = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < np; k += stride) {
    const int2 ab = ws.mpair[k];
    merge_pair(ab.x, ab.y, row_x, c, m, trk, fits, ws, steps);
  }
  // one atomic per wave for the step count
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) steps += __shfl_xor(steps, d);
  if ((threadIdx.x & 63) == 0 && steps) atomicAdd(&ws.counters[kCtrMergeSteps], (unsigned long long)steps);
}

// Link A to its best continuation B when A is B's best predecessor.
__global__ __launch_bounds__(256) void k_merge_link(int S, TracksOut tr, MergeOut out, Workspace ws, int64_t n_max) {
  const int64_t n = min(tr.track_offset[S], n_max);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t A = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; A < n; A += stride) {
    const unsigned long long ka = ws.mkey_a[A];
    if (ka == ~0ull) continue;
    const int32_t B = (int32_t)(ka & 0xffffffffull);
    if ((uint32_t)(ws.mkey_b[B] & 0xffffffffull) != (uint32_t)A) continue;
    out.next[A] = B;
    out.chi2[A] = __uint_as_float((uint32_t)(ka >> 32));
    out.prev[B] = (int32_t)A;
  }
}

// First segment of each chain (rows rise strictly along a chain, so a walk
// is at most R steps).
__global__ __launch_bounds__(256) void k_merge_head(int S, int R, TracksOut tr, MergeOut out, int64_t n_max) {
  const int64_t n = min(tr.track_offset[S], n_max);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
    int32_t h = (int32_t)t;
    for (int i = 0; i < R; ++i) {
      const int32_t p = out.prev[h];
      if (p < 0) break;
      h = p;
    }
    out.head[t] = h;
  }
}

// ------------------------------------------------- binary64-covariance refit
struct MTrk {
  float x, y, z, s, l, q;
  double c00, c10, c11, c20, c21, c22;
  double d00, d10, d11;
};

__device__ __forceinline__ int prop_m(MTrk& t, float x1, float kb) {
  const float dx = x1 - t.x;
  const float k = kb * t.q;
  const float s0 = t.s;
  const float s1 = s0 + k * dx;
  if (!(fabsf(s1) < 0.999f)) return kStepSinPhi;
  // |s0|, |s1| < 0.999 (every state the transport sees passed that check)
  const float c0 = sqrt_unit(1.0f - s0 * s0);
  const float c1 = sqrt_unit(1.0f - s1 * s1);
  const float T = (s0 + s1) / (c0 + c1);
  const float dy = dx * T;
  const float ch = sqrtf(dx * dx + dy * dy);
  const float u = (k * ch) * 0.5f;
  if (!(fabsf(u) <= 0.2f)) return kStepArc;
  const float u2 = u * u;
  const float A = 1.0f + u2 * (1.0f / 6.0f + u2 * (3.0f / 40.0f + u2 * (5.0f / 112.0f + u2 * (35.0f / 1152.0f))));
  float dS = ch * A;
  if (dx < 0.0f) dS = -dS;
  const float sm = (s0 + s1) * 0.5f;
  const float cm2 = 1.0f - sm * sm;
  const float cm3 = cm2 * sqrt_unit(cm2);
  const double a = (double)(dx / cm3);
  const double b = (double)(((kb * dx) * dx * 0.5f) / cm3);
  const double d = (double)(kb * dx);
  const double e = (double)dS;
  t.x = x1;
  t.y = t.y + dy;
  t.z = t.z + t.l * dS;
  t.s = s1;
  const double c00 = t.c00, c10 = t.c10, c11 = t.c11, c20 = t.c20, c21 = t.c21, c22 = t.c22;
  const double m0 = c00 + a * c10 + b * c20;
  const double m1 = c10 + a * c11 + b * c21;
  const double m2 = c20 + a * c21 + b * c22;
  const double n1 = c11 + d * c21;
  const double n2 = c21 + d * c22;
  t.c00 = m0 + a * m1 + b * m2;
  t.c10 = m1 + d * m2;
  t.c11 = n1 + d * n2;
  t.c20 = m2;
  t.c21 = n2;
  const double tz = t.d10 + e * t.d11;
  t.d00 = t.d00 + e * t.d10 + e * tz;
  t.d10 = tz;
  return kStepOk;
}

__device__ __forceinline__ int upd_m(MTrk& t, float my, float mz, double sy2, double sz2) {
  const float ry = my - t.y;
  const double iy = 1.0 / (t.c00 + sy2);
  const double k0 = t.c00 * iy, k1 = t.c10 * iy, k2 = t.c20 * iy;
  t.y = t.y + (float)(k0 * (double)ry);
  t.s = t.s + (float)(k1 * (double)ry);
  t.q = t.q + (float)(k2 * (double)ry);
  const double c00 = t.c00, c10 = t.c10, c20 = t.c20;
  t.c00 = c00 - k0 * c00;
  t.c10 = c10 - k1 * c00;
  t.c20 = c20 - k2 * c00;
  t.c11 = t.c11 - k1 * c10;
  t.c21 = t.c21 - k2 * c10;
  t.c22 = t.c22 - k2 * c20;
  const float rz = mz - t.z;
  const double iz = 1.0 / (t.d00 + sz2);
  const double g0 = t.d00 * iz, g1 = t.d10 * iz;
  t.z = t.z + (float)(g0 * (double)rz);
  t.l = t.l + (float)(g1 * (double)rz);
  const double d00 = t.d00, d10 = t.d10;
  t.d00 = d00 - g0 * d00;
  t.d10 = d10 - g1 * d00;
  t.d11 = t.d11 - g1 * d10;
  return fabsf(t.s) < 0.999f ? kStepOk : kStepSinPhi;
}

__global__ __launch_bounds__(256) void k_refit64(Inputs in, Span sp, int R, const float* __restrict__ row_x,
                                                 Consts c, const int64_t* toff, int64_t first, int64_t cap,
                                                 TrackletOut out) {
  const int64_t lo = max(toff[sp.s0], first);
  const int64_t hi = min(toff[sp.s1], first + cap);
  for (int64_t slot = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; slot < hi;
       slot += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = slot - first;
    const int fl = out.flags[o];
    if (!((c.precision == 1 && (fl & 8)) || c.precision == 2)) continue;
    const int s = sector_of(toff, sp.s0, sp.s1, slot);
    const int64_t a = in.hit_offset[s];
    const int32_t* rh = out.row_hit + o * row_stride(R);
    const int r0 = out.start_row[o];
    MTrk st = {};
    MTrk snap;
    bool ok = r0 >= 0 && r0 + 1 < R && rh[r0] >= 0 && rh[r0 + 1] >= 0;
    if (ok) {
      const int32_t h0 = rh[r0], h1 = rh[r0 + 1];
      const float x0 = row_x[r0], x1 = row_x[r0 + 1];
      const float dx = x1 - x0, dy = in.y[a + h1] - in.y[a + h0], dz = in.z[a + h1] - in.z[a + h0];
      const float L = sqrtf(dx * dx + dy * dy);
      st.x = x0; st.y = in.y[a + h0]; st.z = in.z[a + h0]; st.s = dy / L; st.l = dz / L; st.q = 0.0f;
      st.c00 = c.sy2d; st.c10 = 0.0; st.c11 = 1.0; st.c20 = 0.0; st.c21 = 0.0; st.c22 = 100.0;
      st.d00 = c.sz2d; st.d10 = 0.0; st.d11 = 1.0;
      ok = fabsf(st.s) < 0.999f;
    }
    snap = st;
    if (ok) {
      int lastr = r0, fr = r0;
      for (int r = r0 + 1; r < R; ++r) if (rh[r] >= 0) lastr = r;
      for (int r = r0 - 1; r >= 0; --r) if (rh[r] >= 0) fr = r;
      MTrk last = st;
      int lr = r0;
      for (int r = r0 + 1; r <= lastr; ++r) {
        if (prop_m(st, row_x[r], c.kb)) break;
        if (rh[r] >= 0) {
          MTrk u = st;
          if (upd_m(u, in.y[a + rh[r]], in.z[a + rh[r]], c.sy2d, c.sz2d)) break;
          st = u; last = st; lr = r;
        }
      }
      st = last;
      bool back = true;
      for (int r = lr - 1; r >= r0; --r)
        if (prop_m(st, row_x[r], c.kb)) { back = false; break; }
      snap = back ? st : last;
      if (back) {
        for (int r = r0 - 1; r >= fr; --r) {
          if (prop_m(st, row_x[r], c.kb)) break;
          if (rh[r] >= 0) {
            MTrk u = st;
            if (upd_m(u, in.y[a + rh[r]], in.z[a + rh[r]], c.sy2d, c.sz2d)) break;
            st = u; snap = st;
          }
        }
      }
    }
    out.x_ref[o] = snap.x;
    float* p = out.param + 5 * o;
    p[0] = snap.y; p[1] = snap.z; p[2] = snap.s; p[3] = snap.l; p[4] = snap.q;
    float* cv = out.cov + 15 * o;
    cv[0] = (float)snap.c00; cv[1] = 0.0f; cv[2] = (float)snap.d00; cv[3] = (float)snap.c10; cv[4] = 0.0f;
    cv[5] = (float)snap.c11; cv[6] = 0.0f; cv[7] = (float)snap.d10; cv[8] = 0.0f; cv[9] = (float)snap.d11;
    cv[10] = (float)snap.c20; cv[11] = 0.0f; cv[12] = (float)snap.c21; cv[13] = 0.0f; cv[14] = (float)snap.c22;
    out.flags[o] = fl | 16;
  }
}

// ------------------------------------------------------------------ probe
__global__ void k_fp32_probe(int op, const float* a, const float* b, float* o, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = a[i], y = b[i];
  float r;
  switch (op) {
    case 0: r = x + y; break;
    case 1: r = x - y; break;
    case 2: r = x * y; break;
    case 3: r = x / y; break;
    case 4: r = sqrtf(x); break;
    default: r = sqrt_unit(x); break;
  }
  o[i] = r;
}

// Achievable-peak probes: a 16-byte-per-lane copy, and 8 independent chains
// of binary32 fused multiply-adds per thread.
__global__ __launch_bounds__(256) void k_probe_copy(const int4* __restrict__ src, int4* __restrict__ dst, int64_t n) {
  const int64_t i0 = ((int64_t)blockIdx.x * 256 * 4) + threadIdx.x;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t i = i0 + (int64_t)u * 256;
    if (i < n) dst[i] = src[i];
  }
}

__global__ __launch_bounds__(256) void k_probe_fma(float* out, int64_t n, int iters) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float m = 0.9999999f, c = 1.0e-7f;
  float a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = (float)((i + k) & 1023) * 1.0e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = fmaf(a[k], m, c);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  out[i] = s;
}

inline unsigned blocks_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

// ================================================================ launchers
hipError_t launch_reset(unsigned long long* counters, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, counters, n);
  return hipGetLastError();
}

hipError_t launch_rowk(const float* row_x, int n_rows, float4* rowk, unsigned long long* counters, hipStream_t st) {
  hipLaunchKernelGGL(k_rowk, dim3(blocks_for(n_rows, 256)), dim3(256), 0, st, row_x, n_rows, rowk, counters);
  return hipGetLastError();
}

hipError_t launch_status(const unsigned long long* counters, uint64_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_status, dim3(1), dim3(64), 0, st, counters, status);
  return hipGetLastError();
}

hipError_t launch_row_index(const Inputs& in, Span sp, int n_rows, const float* row_x, const Workspace& ws,
                            int block, hipStream_t st) {
  const int64_t n_items = (int64_t)(sp.s1 - sp.s0) * (n_rows + 1);
  const int64_t item_blocks = blocks_for(n_items, block);
  const int64_t total = item_blocks + blocks_for(sp.h1 - sp.h0, block);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_index, dim3((unsigned)total), dim3(block), 0, st, in, sp, n_rows, row_x, ws.row_first,
                     ws.blk_sec, ws.counters, n_items, item_blocks);
  return hipGetLastError();
}

hipError_t launch_grid(const Inputs& in, Span sp, int n_rows, float bin_hits, const Workspace& ws, hipStream_t st) {
  const int64_t items = (int64_t)(sp.s1 - sp.s0) * n_rows;
  if (items == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grid, dim3((unsigned)items), dim3(64), 0, st, in, sp, n_rows, bin_hits, ws);
  return hipGetLastError();
}

hipError_t launch_neighbours(const Inputs& in, Span sp, int n_rows, const float4* rowk, const Consts& c,
                             const Workspace& ws, int32_t* up, int32_t* dn, int block, int rows, int lds_bytes,
                             hipStream_t st) {
  const int64_t n = sp.h1 - sp.h0;
  if (n == 0) return hipSuccess;
  const int64_t flat_blocks = blocks_for(n, block);
  if (lds_bytes <= 0) {
    hipLaunchKernelGGL(k_nf_flat, dim3((unsigned)flat_blocks), dim3(block), 0, st, in, sp, n_rows, rowk, c, ws, up,
                       dn, flat_blocks);
    return hipGetLastError();
  }
  rows = std::max(1, std::min(rows, kNfMaxRows));  // the workgroup stages the headers of rows + 2 rows
  const int64_t chunks = (n_rows + rows - 1) / rows;
  const int64_t items = (int64_t)(sp.s1 - sp.s0) * chunks;
  hipLaunchKernelGGL(k_neighbours, dim3((unsigned)items), dim3(block), (size_t)lds_bytes, st, in, sp, n_rows, rowk,
                     c, ws, up, dn, rows, lds_bytes);
  return hipGetLastError();
}

hipError_t launch_clean_start(const Inputs& in, Span sp, const int32_t* up, const int32_t* dn, int32_t* up_c,
                              int32_t* dn_c, const Workspace& ws, hipStream_t st) {
  const int64_t n = sp.h1 - sp.h0;
  if (n == 0) return hipSuccess;
  const int64_t nblk = blocks_for(n, kHitsPerBlock);
  hipLaunchKernelGGL(k_clean_start, dim3(blocks_for(nblk, kCleanRounds)), dim3(kHitsPerBlock), 0, st, in, sp, nblk,
                     up, dn, up_c, dn_c, ws);
  return hipGetLastError();
}

hipError_t launch_scan(Span sp, int64_t* toff, const Workspace& ws, hipStream_t st) {
  const int64_t nblk = (sp.h1 - sp.h0 + kHitsPerBlock - 1) / kHitsPerBlock;
  const int64_t ng = nblk / kScanGroup + 1;  // covers entries [0, nblk]
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)ng), dim3(kScanGroup), 0, st, nblk, ws);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, sp, ng, toff, ws);
  return hipGetLastError();
}

hipError_t launch_compact(const Inputs& in, Span sp, int64_t* toff, int32_t* start_hit, const Workspace& ws,
                          hipStream_t st) {
  const int64_t nblk = (sp.h1 - sp.h0 + kHitsPerBlock - 1) / kHitsPerBlock;
  const int64_t word_blocks = blocks_for(nblk * (kHitsPerBlock / 64), kHitsPerBlock);
  const int64_t nsec_blk = ((int64_t)(sp.s1 - sp.s0) + kHitsPerBlock - 1) / kHitsPerBlock;
  const int64_t grid = word_blocks + nsec_blk;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact, dim3((unsigned)grid), dim3(kHitsPerBlock), 0, st, in, sp, nblk, word_blocks, toff,
                     start_hit, ws);
  return hipGetLastError();
}

hipError_t launch_tracklets(const Inputs& in, Span sp, int n_rows, const float* row_x, const Consts& c,
                            const Workspace& ws, const int64_t* toff, int64_t first, int64_t cap,
                            const TrackletOut& out, int grid, int block, int nparts, int waves, int sync,
                            hipStream_t st) {
  const int S = sp.s1 - sp.s0;
  if (S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batches, dim3(1), dim3(1024), 0, st, toff, sp.s0, sp.s1, ws.batch_off);
  const size_t lds = (size_t)tc_planes_bytes(n_rows) + (sync ? (size_t)(block / 64) * kStageBytes : 0);
#define CATPC_TC(K)                                                                                           \
  do {                                                                                                        \
    if (sync)                                                                                                 \
      hipLaunchKernelGGL((k_tracklets<K, true>), dim3(grid), dim3(block), lds, st, in, sp, n_rows, row_x, c, ws, \
                         toff, first, cap, out, nparts);                                                      \
    else                                                                                                      \
      hipLaunchKernelGGL((k_tracklets<K, false>), dim3(grid), dim3(block), lds, st, in, sp, n_rows, row_x, c,    \
                         ws, toff, first, cap, out, nparts);                                                  \
  } while (0)
  switch (waves) {
    case 5: CATPC_TC(5); break;
    case 6: CATPC_TC(6); break;
    case 8: CATPC_TC(8); break;
    default: CATPC_TC(0); break;
  }
#undef CATPC_TC
  return hipGetLastError();
}

hipError_t launch_select(const Inputs& in, int S, const int64_t* toff, int64_t cap, int64_t max_slots, int n_rows,
                         const TrackletOut& trk, const Consts& c, const Workspace& ws, const TracksOut& out,
                         int64_t n_hits, int grid, hipStream_t st) {
  const int64_t slots = std::min(cap, max_slots);
  const int64_t ng = slots / kScanGroup + 1;  // covers entries [0, slots]
  (void)n_hits;
  hipLaunchKernelGGL(k_sel_flags, dim3(1), dim3(64), 0, st, ws);
  const int64_t claim_blocks = (int64_t)S * sel_chunks(n_rows);
  if (claim_blocks > 0)
    hipLaunchKernelGGL(k_sel_claim, dim3((unsigned)claim_blocks), dim3(256), 0, st, in, S, toff, slots, n_rows, trk,
                       ws);
  hipLaunchKernelGGL(k_sel_count, dim3(grid), dim3(256), 0, st, toff, S, slots, n_rows, trk, c, ws);
  hipLaunchKernelGGL(k_sel_scan_local, dim3((unsigned)ng), dim3(kScanGroup), 0, st, toff, S, slots, ws);
  hipLaunchKernelGGL(k_sel_scan_top, dim3(1), dim3(1024), 0, st, ng, ws);
  hipLaunchKernelGGL(k_sel_emit, dim3(grid), dim3(256), 0, st, in, S, toff, slots, n_rows, trk, ws, out);
  return hipGetLastError();
}

hipError_t launch_fullfit(const Inputs& in, int S, int n_rows, const float* row_x, const Consts& c,
                          const int64_t* toff, const TrackletOut& trk, int64_t trk_cap, const TracksOut& tr,
                          const FitsOut& out, const Workspace& ws, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_fullfit, dim3(grid), dim3(256), sizeof(float) * (size_t)n_rows, st, in, S, n_rows, row_x, c,
                     toff, trk, trk_cap, tr, out, ws);
  return hipGetLastError();
}

hipError_t launch_merge(const Inputs& in, int S, int n_rows, const float* row_x, const Consts& c,
                        const MergeCuts& m, const int64_t* toff, const TrackletOut& trk, int64_t trk_cap,
                        const TracksOut& tr, const FitsOut& fits, const MergeOut& out, const Workspace& ws,
                        int64_t max_slots, int grid, int pair_grid, int64_t pair_cap, hipStream_t st) {
  const int64_t n_max = std::min(std::min(tr.track_capacity, fits.capacity), std::min(out.capacity, max_slots));
  pair_cap = std::max<int64_t>(0, std::min(pair_cap, kMergePairsPerSlot * max_slots));
  hipLaunchKernelGGL(k_merge_prep, dim3(grid), dim3(256), 0, st, in, S, n_rows, toff, trk, trk_cap, tr, fits, out,
                     ws, n_max);
  hipLaunchKernelGGL(k_merge_chunks, dim3(1), dim3(1024), 0, st, S, tr, ws, n_max);
  hipLaunchKernelGGL(k_merge_cand, dim3((unsigned)pair_grid), dim3(256), 0, st, S, m, tr, fits, ws, n_max, pair_cap);
  hipLaunchKernelGGL(k_merge_chi2, dim3(pair_grid), dim3(256), 0, st, S, row_x, c, m, toff, trk, tr, fits, ws,
                     pair_cap);
  hipLaunchKernelGGL(k_merge_over, dim3(grid), dim3(256), 0, st, S, row_x, c, m, toff, trk, tr, fits, ws, n_max);
  hipLaunchKernelGGL(k_merge_link, dim3(grid), dim3(256), 0, st, S, tr, out, ws, n_max);
  hipLaunchKernelGGL(k_merge_head, dim3(grid), dim3(256), 0, st, S, n_rows, tr, out, n_max);
  return hipGetLastError();
}

hipError_t launch_refit64(const Inputs& in, Span sp, int n_rows, const float* row_x, const Consts& c,
                          const Workspace& ws, const int64_t* toff, int64_t first, int64_t cap,
                          const TrackletOut& out, int grid, hipStream_t st) {
  (void)ws;
  hipLaunchKernelGGL(k_refit64, dim3(grid), dim3(256), 0, st, in, sp, n_rows, row_x, c, toff, first, cap, out);
  return hipGetLastError();
}

hipError_t launch_probe_copy(const void* src, void* dst, int64_t n16, hipStream_t st) {
  if (n16 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_probe_copy, dim3(blocks_for(n16, 256 * 4)), dim3(256), 0, st, (const int4*)src, (int4*)dst, n16);
  return hipGetLastError();
}

hipError_t launch_probe_fma(float* out, int64_t n, int iters, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_probe_fma, dim3(blocks_for(n, 256)), dim3(256), 0, st, out, n, iters);
  return hipGetLastError();
}

hipError_t phase_clocks(unsigned long long* out, bool clear) {
  if (!kPhaseClocks) return hipErrorNotSupported;
  if (clear) {
    const unsigned long long z[kPhaseSlots] = {};
    return hipMemcpyToSymbol(HIP_SYMBOL(g_phase_clocks), z, sizeof(z));
  }
  return hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase_clocks), sizeof(unsigned long long) * kPhaseSlots);
}

hipError_t launch_fp32_probe(int op, const float* a, const float* b, float* out, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fp32_probe, dim3(blocks_for(n, 256)), dim3(256), 0, st, op, a, b, out, n);
  return hipGetLastError();
}

}  // namespace catpc
