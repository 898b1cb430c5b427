// HIP kernels (gfx950) for continuous sensor registration.
//
// Hot path, per gradient-flow iteration (launches shared by all active
// requests of one kernel variant):
//   k_prepare  one wavefront per cluster of <= 64 spatially sorted targets:
//              z~_j = T z_j in FP64, the cluster frame (origin, scaled
//              relative targets, bounding box), the compacted list of
//              reachable non-empty source cells of the current length-scale
//              grid, and the cut of the cluster's candidates into work items.
//   k_pairs    persistent workgroups over the work items: each item's
//              candidate sources are culled against the cluster box, staged
//              in the wave's LDS area and paired with the cluster's targets
//              (one per lane), FP32 pair terms
//                  d = z~_j - x_i, r^2, e = exp(-r^2/(2 l^2)), c = <l_i, m_j>,
//                  W_j += c e, D_j += c e d          (eq. scalar, eq. 3_gradient)
//              with compensated (Kahan) FP32 partials per lane and an FP64
//              wave reduction into the item's row.
//   k_reduce   one wavefront per cluster: the cluster's item rows, in order.
//   k_step     one block per request: a fixed FP64 reduction tree over the
//              cluster rows, F, omega, v and the FP64 exponential-map step
//              (eq. step, eq. newstep) applied to the pose.
// With the quartic step rule (Sec. VI-B, eq. fourth) k_step first stores the
// gradient only; a second k_pairs pass over the same items sums the Taylor
// coefficients A1..A4 of G(t) = F(h exp(t xi)) along it, and a second
// k_reduce / k_step pair takes the maximiser of the quartic as the step.
//
// Set-up kernels (once per registration): bounding boxes and the default
// a^2 (FP64), one source grid per length-scale stage (deterministic counting
// sort by cell), a Morton order of the targets and its clusters.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <atomic>
#include <type_traits>

#include "cvo_internal.h"
#include "cvo_step.h"

namespace cvo {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename P>
__device__ __forceinline__ P* uniform_ptr(P* p) {
  const unsigned long long u = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return (P*)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ double uniform_d(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Cross-lane reductions on DPP row operations (no LDS traffic): within each
// row of 16 lanes, xor-1 and xor-2 quad permutations, then the half-row and
// row mirrors give every lane its row's result; the four row results are
// read as scalars and combined in a fixed order.  Every lane returns the same
// value, and the association is fixed, so results are reproducible.
template <int CTRL>
__device__ __forceinline__ int dpp32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)dpp32<CTRL>((int)(unsigned)u);
  const unsigned hi = (unsigned)dpp32<CTRL>((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;
constexpr int kDppRowShr = 0x110;     // + n: row_shr:n
constexpr int kDppBcast15 = 0x142;
constexpr int kDppBcast31 = 0x143;

template <typename Op>
__device__ __forceinline__ double wave_reduce_d(double v, Op op) {
  v = op(v, dpp64<kDppXor1>(v));
  v = op(v, dpp64<kDppXor2>(v));
  v = op(v, dpp64<kDppHalfMirror>(v));
  v = op(v, dpp64<kDppMirror>(v));
  return op(op(readlane_d(v, 0), readlane_d(v, 16)), op(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ double wave_sum(double v) {
  return wave_reduce_d(v, [](double a, double b) { return a + b; });
}
__device__ __forceinline__ double wave_min(double v) {
  return wave_reduce_d(v, [](double a, double b) { return fmin(a, b); });
}
__device__ __forceinline__ double wave_max(double v) {
  return wave_reduce_d(v, [](double a, double b) { return fmax(a, b); });
}
__device__ __forceinline__ int wave_sum_int(int v) {
  v += dpp32<kDppXor1>(v);
  v += dpp32<kDppXor2>(v);
  v += dpp32<kDppHalfMirror>(v);
  v += dpp32<kDppMirror>(v);
  return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
         (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}
// inclusive prefix sum over the wave: Hillis-Steele inside each row of 16
// (row shifts, zero fill), then the row totals are carried by the row
// broadcasts of lanes 15 and 31
__device__ __forceinline__ int wave_incl_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr + 1, 0xF, 0xF, true);
  v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr + 2, 0xF, 0xF, true);
  v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr + 4, 0xF, 0xF, true);
  v += __builtin_amdgcn_update_dpp(0, v, kDppRowShr + 8, 0xF, 0xF, true);
  v += __builtin_amdgcn_update_dpp(0, v, kDppBcast15, 0xA, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, v, kDppBcast31, 0xC, 0xF, false);
  return v;
}
// value of a wave-uniform lane index, as a scalar
__device__ __forceinline__ int lane_value(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// ---------------------------------------------------------------------------
// 1) bounding box and mean squared norm (FP64), two passes
//    partial layout per block: min xyz, max xyz, sum |p|^2
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bbox_partial(const float* __restrict__ xyz, int n,
                                                      double* __restrict__ part) {
  __shared__ double sh[7][256];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY}, s2 = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double p[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
    for (int a = 0; a < 3; a++) {
      mn[a] = fmin(mn[a], p[a]);
      mx[a] = fmax(mx[a], p[a]);
    }
    s2 += p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  }
  const int t = threadIdx.x;
  for (int a = 0; a < 3; a++) {
    sh[a][t] = mn[a];
    sh[3 + a][t] = mx[a];
  }
  sh[6][t] = s2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      for (int a = 0; a < 3; a++) {
        sh[a][t] = fmin(sh[a][t], sh[a][t + o]);
        sh[3 + a][t] = fmax(sh[3 + a][t], sh[3 + a][t + o]);
      }
      sh[6][t] += sh[6][t + o];
    }
    __syncthreads();
  }
  if (t < 7) part[7 * blockIdx.x + t] = sh[t][0];
}

// out: min xyz, max xyz, mean |p|^2.  One block of kBboxThreads: thread t
// folds partials t, t + kBboxThreads, ... in order, then a fixed tree in LDS
// (the same order on every run).
constexpr int kBboxThreads = 256;
__global__ __launch_bounds__(kBboxThreads) void k_bbox_final(const double* __restrict__ part, int nblk, int n,
                                                            double* __restrict__ out) {
  __shared__ double sh[7][kBboxThreads];
  const int t = threadIdx.x;
  double r[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
  for (int b = t; b < nblk; b += kBboxThreads) {
    for (int a = 0; a < 3; a++) {
      r[a] = fmin(r[a], part[7 * b + a]);
      r[3 + a] = fmax(r[3 + a], part[7 * b + 3 + a]);
    }
    r[6] += part[7 * b + 6];
  }
  for (int q = 0; q < 7; q++) sh[q][t] = r[q];
  __syncthreads();
  for (int o = kBboxThreads / 2; o > 0; o >>= 1) {
    if (t < o) {
      for (int a = 0; a < 3; a++) {
        sh[a][t] = fmin(sh[a][t], sh[a][t + o]);
        sh[3 + a][t] = fmax(sh[3 + a][t], sh[3 + a][t + o]);
      }
      sh[6][t] += sh[6][t + o];
    }
    __syncthreads();
  }
  if (t < 7) out[t] = (t == 6) ? sh[6][0] / (double)n : sh[t][0];
}

// ---------------------------------------------------------------------------
// 2) grid geometry for every stage (one thread per stage)
//    cell edge: kappa*ell/cells_per_reach with the cutoff, else a coarse edge
//    (extent/brute_div) used only for cell-local precision.  The edge grows
//    if the dense table would exceed kcap cells.
// ---------------------------------------------------------------------------
__global__ void k_grid_setup(const double* __restrict__ xbox, int n_stages, const double* __restrict__ ells,
                             double kappa, int cells_per_reach, int brute_div, int kcap,
                             GridInfo* __restrict__ grid, int* __restrict__ ncell_out) {
  const int s = threadIdx.x;
  if (blockIdx.x != 0) return;
  if (s == 0) ncell_out[n_stages] = kZBuckets;  // key range of the target order
  if (s >= n_stages) return;
  const double ell = ells[s];
  const double lo[3] = {xbox[0], xbox[1], xbox[2]};
  double ext[3];
  double emax = 0.0;
  for (int a = 0; a < 3; a++) {
    ext[a] = fmax(xbox[3 + a] - lo[a], 0.0);
    emax = fmax(emax, ext[a]);
  }
  // non-finite or absurd extents only occur for inputs that the finiteness
  // check rejects; keep the geometry well defined (one cell) for them
  if (!isfinite(emax) || emax > 1e12 || !isfinite(lo[0] + lo[1] + lo[2])) {
    for (int a = 0; a < 3; a++) ext[a] = 0.0;
    emax = 0.0;
  }
  GridInfo g;
  g.cutoff = kappa > 0.0 ? 1 : 0;
  double h;
  if (g.cutoff) {
    h = kappa * ell / (double)cells_per_reach;
  } else {
    h = fmax(emax / (double)brute_div, 1e-3);
  }
  if (!(h > 0.0)) h = 1.0;
  int dims[3] = {1, 1, 1};
  bool fits = false;
  for (int it = 0; it < 256 && !fits; it++) {
    double cells = 1.0;
    bool axis_ok = true;
    for (int a = 0; a < 3; a++) {
      const double d = floor(ext[a] / h) + 1.0;
      cells *= d;
      axis_ok = axis_ok && d <= (double)kMaxDim;
    }
    if (cells <= (double)kcap && axis_ok) fits = true;
    else h *= 1.25;
  }
  if (!fits) h = 2.0 * emax + 1.0;  // at most 8 cells
  for (int a = 0; a < 3; a++) dims[a] = (int)floor(ext[a] / h) + 1;
  const bool finite_lo = isfinite(lo[0] + lo[1] + lo[2]);
  g.ox = finite_lo ? lo[0] : 0.0;
  g.oy = finite_lo ? lo[1] : 0.0;
  g.oz = finite_lo ? lo[2] : 0.0;
  g.h = h;
  g.nx = dims[0];
  g.ny = dims[1];
  g.nz = dims[2];
  g.ncell = dims[0] * dims[1] * dims[2];
  g.ell = ell;
  const double LOG2E = 1.4426950408889634074;
  g.sq = sqrt(LOG2E / (2.0 * ell * ell));
  if (g.cutoff) {
    // kappa^2 ell^2 * log2(e)/(2 ell^2)
    g.rc2s = kappa * kappa * LOG2E * 0.5;
    // candidate cells must contain every source the FP32 test can accept
    g.reach = kappa * ell * (1.0 + 1e-5) + 1e-7;
  } else {
    g.rc2s = INFINITY;
    g.reach = 0.0;
  }
  g.pad = 0;
  grid[s] = g;
  ncell_out[s] = g.ncell;
}

// ---------------------------------------------------------------------------
// 3) keys
// ---------------------------------------------------------------------------
// cell index of coordinate u (in cell units), clamped to [0, dim-1] before
// the conversion; non-finite u maps to cell 0
__device__ __forceinline__ int cell_of(double u, int dim) {
  if (!isfinite(u)) return 0;
  return (int)fmin(fmax(floor(u), 0.0), (double)(dim - 1));
}

// source cell keys for every stage (blockIdx.y = stage)
__global__ __launch_bounds__(256) void k_src_keys(const float* __restrict__ xyz, int n,
                                                  const GridInfo* __restrict__ grid, int* __restrict__ keys) {
  const int s = blockIdx.y;
  const GridInfo g = grid[s];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    const int cx = cell_of((x - g.ox) / g.h, g.nx);
    const int cy = cell_of((y - g.oy) / g.h, g.ny);
    const int cz = cell_of((z - g.oz) / g.h, g.nz);
    keys[(size_t)s * n + i] = (cz * g.ny + cy) * g.nx + cx;
  }
}

__device__ __forceinline__ unsigned spread3(unsigned v) {  // 10 bits -> every third bit
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Morton key of the target points on a 2^kZBits grid over their bounding box
__global__ __launch_bounds__(256) void k_tgt_keys(const float* __restrict__ xyz, int m,
                                                  const double* __restrict__ zbox, int* __restrict__ keys) {
  const double res = (double)(1 << kZBits);
  double lo[3], inv[3];
  for (int a = 0; a < 3; a++) {
    lo[a] = zbox[a];
    const double e = zbox[3 + a] - zbox[a];
    inv[a] = (e > 0.0 && isfinite(e)) ? res / e : 0.0;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    unsigned c[3];
    for (int a = 0; a < 3; a++) {
      const double u = ((double)xyz[3 * i + a] - lo[a]) * inv[a];
      c[a] = (unsigned)cell_of(u, 1 << kZBits);
    }
    keys[i] = (int)(spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2));
  }
}

// ---------------------------------------------------------------------------
// 4) stable key sort (blockIdx.y = segment): least-significant-digit radix
//    sort over 8-bit digits.  Pass p: per block of kRadixTile consecutive
//    elements (of the previous pass's order) the digit counts; their
//    exclusive scan in digit-major order gives each (digit, block) its first
//    output position; the scatter gives each element its rank among the
//    equal digits of its block in element order.  Every pass is stable and
//    the first one starts in index order, so the result is the order by key
//    with ties by index, independent of scheduling.  The start table is found
//    from the sorted keys by binary search.
// ---------------------------------------------------------------------------
__device__ __forceinline__ const int* radix_keys_in(const SortSeg& S, int pass) {
  return pass == 0 ? S.keys : (((pass - 1) & 1) ? S.key_b : S.key_a);
}

__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const SortSeg* __restrict__ segs, int pass) {
  static_assert(kRadixThreads == kRadixBins, "one digit per thread");
  const SortSeg S = segs[blockIdx.y];
  const int b = blockIdx.x;
  if (b >= S.nblocks) return;  // block-uniform
  __shared__ int h[kRadixBins];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const int* __restrict__ keys = radix_keys_in(S, pass);
  const int shift = 8 * pass;
  for (int e = 0; e < kRadixRounds; e++) {
    const int i = b * kRadixTile + e * kRadixThreads + t;
    if (i < S.n) atomicAdd(&h[(keys[i] >> shift) & (kRadixBins - 1)], 1);
  }
  __syncthreads();
  S.hist[(size_t)t * S.nblocks + b] = h[t];
}

__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const SortSeg* __restrict__ segs, int pass,
                                                                  int last) {
  constexpr int NW = kRadixThreads / kWave;
  const SortSeg S = segs[blockIdx.y];
  const int b = blockIdx.x;
  if (b >= S.nblocks) return;  // block-uniform
  __shared__ int base[kRadixBins];     // next output position of each digit in this block
  __shared__ int wpos[NW][kRadixBins]; // per round: the waves' counts, then their first positions
  const int t = threadIdx.x, w = t >> 6, l = lane_id();
  base[t] = S.hist[(size_t)t * S.nblocks + b];
  const int* __restrict__ ksrc = radix_keys_in(S, pass);
  const int* __restrict__ isrc = pass == 0 ? nullptr : (((pass - 1) & 1) ? S.idx_b : S.idx_a);
  int* __restrict__ kdst = (pass & 1) ? S.key_b : S.key_a;
  int* __restrict__ idst = last ? S.perm : ((pass & 1) ? S.idx_b : S.idx_a);
  const int shift = 8 * pass;
  const unsigned long long below = (1ull << l) - 1ull;  // lanes 0 .. l-1
  for (int e = 0; e < kRadixRounds; e++) {
#pragma unroll
    for (int ww = 0; ww < NW; ww++) wpos[ww][t] = 0;
    __syncthreads();
    const int i = b * kRadixTile + e * kRadixThreads + t;
    const bool valid = i < S.n;
    const int key = valid ? ksrc[i] : 0;
    const int idx = valid ? (pass == 0 ? i : isrc[i]) : 0;
    const int d = (key >> shift) & (kRadixBins - 1);
    // lanes of this wave with the same digit
    unsigned long long same = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; bit++) {
      const bool on = (d >> bit) & 1;
      const unsigned long long bb = __ballot(on);
      same &= on ? bb : ~bb;
    }
    const int rank = __popcll(same & below);
    if (valid && rank == 0) wpos[w][d] = __popcll(same);
    __syncthreads();
    // digit t: the waves' first positions in wave order, and the next round's base
    int run = base[t];
#pragma unroll
    for (int ww = 0; ww < NW; ww++) {
      const int c = wpos[ww][t];
      wpos[ww][t] = run;
      run += c;
    }
    base[t] = run;
    __syncthreads();
    if (valid) {
      const int pos = wpos[w][d] + rank;
      kdst[pos] = key;
      idst[pos] = idx;
    }
    __syncthreads();
  }
}

// start table: count[k] = first sorted position with key >= k, k = 0..K
__global__ __launch_bounds__(256) void k_radix_start(const SortSeg* __restrict__ segs, int passes) {
  const SortSeg S = segs[blockIdx.y];
  const int K = *S.nkeys;
  const int* __restrict__ sk = ((passes - 1) & 1) ? S.key_b : S.key_a;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= K; k += gridDim.x * blockDim.x) {
    int lo = 0, hi = S.n;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sk[mid] < k) lo = mid + 1;
      else hi = mid;
    }
    S.count[k] = lo;
  }
}

// ---------------------------------------------------------------------------
// 5) records
// ---------------------------------------------------------------------------
// target records: raw xyz + labels in Morton order, plus the original index
__global__ __launch_bounds__(256) void k_tgt_records(const float* __restrict__ xyz, const float* __restrict__ feat,
                                                     int m, int fd, int zs, const int* __restrict__ perm,
                                                     float* __restrict__ zrec, int* __restrict__ zorig) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
    const int j = perm[p];
    float* r = zrec + (size_t)p * zs;
    r[0] = xyz[3 * j];
    r[1] = xyz[3 * j + 1];
    r[2] = xyz[3 * j + 2];
    for (int f = 0; f < zs - 3; f++) r[3 + f] = (f < fd) ? feat[(size_t)fd * j + f] : 0.0f;
    zorig[p] = j;
  }
}

// source records per stage (blockIdx.y): scaled offsets from the cell corner + labels
template <typename CT>
__global__ __launch_bounds__(256) void k_src_records(const float* __restrict__ xyz, const float* __restrict__ feat,
                                                     int n, int fd, int xs, const GridInfo* __restrict__ grid,
                                                     const int* __restrict__ keys, const int* __restrict__ perms,
                                                     CT* const* __restrict__ xrec) {
  const int s = blockIdx.y;
  const GridInfo g = grid[s];
  const int* perm = perms + (size_t)s * n;
  const int* key = keys + (size_t)s * n;
  CT* out = xrec[s];
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    const int i = perm[p];
    const int k = key[i];
    const int cx = k % g.nx, cy = (k / g.nx) % g.ny, cz = k / (g.nx * g.ny);
    CT* r = out + (size_t)p * xs;
    r[0] = (CT)(((double)xyz[3 * i] - (g.ox + cx * g.h)) * g.sq);
    r[1] = (CT)(((double)xyz[3 * i + 1] - (g.oy + cy * g.h)) * g.sq);
    r[2] = (CT)(((double)xyz[3 * i + 2] - (g.oz + cz * g.h)) * g.sq);
    for (int f = 0; f < xs - 3; f++) r[3 + f] = (f < fd) ? (CT)feat[(size_t)fd * i + f] : (CT)0;
  }
}


// ---------------------------------------------------------------------------
// multi-block exclusive scan (in place), batched over segments (blockIdx.y)
//   up:   per-tile totals      mid: scan of the tile totals      down: apply
// ---------------------------------------------------------------------------

__device__ __forceinline__ int scan_len(const ScanArgs& A) { return (A.lenp ? *A.lenp : 0) + A.len0; }

// exclusive scan of one value per thread over a 1024-thread block
__device__ __forceinline__ int block_excl_scan(int v, int* sh, int& total) {
  const int l = lane_id(), w = threadIdx.x >> 6;
  const int incl = wave_incl_scan(v);
  if (l == kWave - 1) sh[w] = incl;
  __syncthreads();
  if (w == 0) {
    const int nw = blockDim.x / kWave;
    const int t = (l < nw) ? sh[l] : 0;
    const int ti = wave_incl_scan(t);
    if (l < nw) sh[l] = ti - t;
    if (l == nw - 1) sh[32] = ti;
  }
  __syncthreads();
  total = sh[32];
  const int r = sh[w] + incl - v;
  __syncthreads();
  return r;
}

// the whole scan in one block when it fits one tile
__global__ __launch_bounds__(kScanBlock) void k_scan_single(const ScanArgs* __restrict__ args) {
  const ScanArgs A = args[blockIdx.y];
  const int len = scan_len(A);
  const long long t0 = (long long)threadIdx.x * kScanPerThread;
  int v[kScanPerThread];
  int s = 0;
  for (int k = 0; k < kScanPerThread; k++) {
    v[k] = (t0 + k < len) ? A.data[t0 + k] : 0;
    s += v[k];
  }
  __shared__ int sh[33];
  int total;
  int run = block_excl_scan(s, sh, total);
  for (int k = 0; k < kScanPerThread; k++) {
    if (t0 + k < len) A.data[t0 + k] = run;
    run += v[k];
  }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_up(const ScanArgs* __restrict__ args) {
  const ScanArgs A = args[blockIdx.y];
  const int len = scan_len(A);
  const long long base = (long long)blockIdx.x * kScanTile;
  if (base >= len) return;
  const long long t0 = base + (long long)threadIdx.x * kScanPerThread;
  int s = 0;
  for (int k = 0; k < kScanPerThread; k++)
    if (t0 + k < len) s += A.data[t0 + k];
  __shared__ int sh[33];
  int total;
  (void)block_excl_scan(s, sh, total);
  if (threadIdx.x == 0) A.sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_mid(const ScanArgs* __restrict__ args) {
  const ScanArgs A = args[blockIdx.y];
  const int len = scan_len(A);
  const int nt = (len + kScanTile - 1) / kScanTile;  // <= kScanBlock (checked on the host)
  const int t = threadIdx.x;
  const int v = (t < nt) ? A.sums[t] : 0;
  __shared__ int sh[33];
  int total;
  const int e = block_excl_scan(v, sh, total);
  if (t < nt) A.sums[t] = e;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_down(const ScanArgs* __restrict__ args) {
  const ScanArgs A = args[blockIdx.y];
  const int len = scan_len(A);
  const long long base = (long long)blockIdx.x * kScanTile;
  if (base >= len) return;
  const long long t0 = base + (long long)threadIdx.x * kScanPerThread;
  int v[kScanPerThread];
  int s = 0;
  for (int k = 0; k < kScanPerThread; k++) {
    v[k] = (t0 + k < len) ? A.data[t0 + k] : 0;
    s += v[k];
  }
  __shared__ int sh[33];
  int total;
  int run = block_excl_scan(s, sh, total) + A.sums[blockIdx.x];
  for (int k = 0; k < kScanPerThread; k++) {
    if (t0 + k < len) A.data[t0 + k] = run;
    run += v[k];
  }
}

// ---------------------------------------------------------------------------
// target clusters, one clustering per length-scale stage: runs of at most 64
// consecutive Morton-ordered targets, cut (with a cutoff) wherever two
// consecutive targets are farther apart than D = max(2.5 Morton bucket
// edges, 2 x the stage's cutoff radius), so that no cluster straddles a large
// jump of the Morton curve.
// ---------------------------------------------------------------------------
// (blockIdx.y = stage in all of them; scratch and outputs [stage][m])
__global__ __launch_bounds__(256) void k_cl_flags(const float* __restrict__ zrec, int zs, int m,
                                                  const double* __restrict__ zbox, double kappa,
                                                  const double* __restrict__ stage_ell,
                                                  int* __restrict__ flag_all, int* __restrict__ scan_all) {
  const int stage = blockIdx.y;
  int* __restrict__ flag = flag_all + (size_t)stage * m;
  int* __restrict__ scan = scan_all + (size_t)stage * m;
  double e = 0.0;
  for (int a = 0; a < 3; a++) e = fmax(e, zbox[3 + a] - zbox[a]);
  // with a cutoff, a gap up to twice the cutoff radius stays inside a cluster:
  // fuller clusters (fewer idle lanes) cost fewer candidate slots than the
  // larger boxes add, while the cutoff is large against the Morton buckets
  // Without a cutoff every source pairs with every target: no gap cuts at
  // all (runs of 64 in Morton order), or a sparse cloud would fall apart into
  // clusters of a few targets and leave most lanes idle.
  const double D = fmax(2.5 * e / (double)(1 << kZBits), 2.0 * kappa * stage_ell[stage]);
  const double D2 = isfinite(D) ? D * D : 0.0;
  const bool gaps = kappa > 0.0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
    int f = p == 0 ? 1 : 0;
    if (p > 0 && gaps) {
      const float* a = zrec + (size_t)p * zs;
      const float* b = zrec + (size_t)(p - 1) * zs;
      const double dx = (double)a[0] - b[0], dy = (double)a[1] - b[1], dz = (double)a[2] - b[2];
      f = (dx * dx + dy * dy + dz * dz > D2) ? 1 : 0;
    }
    flag[p] = f;
    scan[p] = f;
  }
}

// segment of p = (exclusive flag scan at p) + flag[p] - 1; record segment starts
__global__ __launch_bounds__(256) void k_cl_segfirst(const int* __restrict__ flag_all, const int* __restrict__ scan_all,
                                                     int m, int* __restrict__ first_all) {
  const size_t so = (size_t)blockIdx.y * m;
  const int* __restrict__ flag = flag_all + so;
  const int* __restrict__ scan = scan_all + so;
  int* __restrict__ first = first_all + so;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x)
    if (flag[p]) first[scan[p]] = p;
}

// cluster-start flags: a segment start, or every 64th target inside a segment
__global__ __launch_bounds__(256) void k_cl_cflags(int* __restrict__ flag_all, int* __restrict__ scan_all,
                                                   const int* __restrict__ first_all, int m) {
  const size_t so = (size_t)blockIdx.y * m;
  int* __restrict__ flag = flag_all + so;
  int* __restrict__ scan = scan_all + so;
  const int* __restrict__ first = first_all + so;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
    const int seg = scan[p] + flag[p] - 1;
    const int pos = p - first[seg];
    const int c = (pos % kWave == 0) ? 1 : 0;
    flag[p] = c;
    scan[p] = c;
  }
}

__global__ __launch_bounds__(256) void k_cl_table(const int* __restrict__ cflag_all, const int* __restrict__ cscan_all,
                                                  int m, int* __restrict__ clus_start_all,
                                                  ReqState* __restrict__ S) {
  const int stage = blockIdx.y;
  const size_t so = (size_t)stage * m;
  const int* __restrict__ cflag = cflag_all + so;
  const int* __restrict__ cscan = cscan_all + so;
  int* __restrict__ clus_start = clus_start_all + so;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x) {
    if (cflag[p]) clus_start[cscan[p]] = p;
    if (p == m - 1) S->nclus_s[stage] = cscan[p] + cflag[p];
  }
}

__global__ __launch_bounds__(256) void k_cl_count(const int* __restrict__ clus_start_all,
                                                  const ReqState* __restrict__ S, int m,
                                                  int* __restrict__ clus_count_all) {
  const int stage = blockIdx.y;
  const int* __restrict__ clus_start = clus_start_all + (size_t)stage * m;
  int* __restrict__ clus_count = clus_count_all + (size_t)stage * m;
  const int nc = S->nclus_s[stage];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x)
    clus_count[c] = ((c + 1 < nc) ? clus_start[c + 1] : m) - clus_start[c];
}

// The mutable states of a launch's requests, copied next to each other so
// that the host reads them back with one copy (request k -> out[k]).
__global__ __launch_bounds__(256) void k_gather_states(const ReqStatic* __restrict__ reqs, int nreq,
                                                       ReqState* __restrict__ out) {
  static_assert(sizeof(ReqState) % 8 == 0, "states are copied as 8-byte words");
  constexpr int W = (int)(sizeof(ReqState) / 8);
  const long long total = (long long)nreq * W;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(i / W), w = (int)(i % W);
    ((unsigned long long*)(out + k))[w] = ((const unsigned long long*)reqs[k].state)[w];
  }
}

__global__ __launch_bounds__(256) void k_zero(unsigned* __restrict__ p, size_t words) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ---------------------------------------------------------------------------
// pair terms
// ---------------------------------------------------------------------------
template <typename CT>
struct Acc;  // per-lane accumulators of W and D

template <>
struct Acc<float> {
  // block sums (plain FP32 over at most kBlock pairs) folded into Kahan pairs
  float w, dx, dy, dz;
  float sw, sx, sy, sz;  // compensated sums
  float cw, cx, cy, cz;  // compensations
  __device__ void init() { w = dx = dy = dz = sw = sx = sy = sz = cw = cx = cy = cz = 0.0f; }
  __device__ static void kahan(float& s, float& c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ void fold() {
    kahan(sw, cw, w);
    kahan(sx, cx, dx);
    kahan(sy, cy, dy);
    kahan(sz, cz, dz);
    w = dx = dy = dz = 0.0f;
  }
  __device__ void result(double& W, double& X, double& Y, double& Z) {
    fold();
    W = (double)sw - (double)cw;
    X = (double)sx - (double)cx;
    Y = (double)sy - (double)cy;
    Z = (double)sz - (double)cz;
  }
};

template <>
struct Acc<double> {
  double w, dx, dy, dz;
  __device__ void init() { w = dx = dy = dz = 0.0; }
  __device__ void fold() {}
  __device__ void result(double& W, double& X, double& Y, double& Z) {
    W = w;
    X = dx;
    Y = dy;
    Z = dz;
  }
};

__device__ __forceinline__ float kexp2(float a) { return __builtin_amdgcn_exp2f(a); }
__device__ __forceinline__ double kexp2(double a) { return exp2(a); }

constexpr int kBlock = 64;  // pairs per lane between Kahan folds

// Source records are read through the constant address space with a
// wave-uniform index, so they arrive in scalar registers (s_load) and every
// lane pairs the same source with its own target.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename CT, int FD, bool CUT>
__device__ __forceinline__ void one_pair(const CT* __restrict__ r, CT zx, CT zy, CT zz, const CT (&mj)[FD], CT rc2,
                                         Acc<CT>& acc, unsigned int& within_blk) {
  const CT dx = zx - r[0];
  const CT dy = zy - r[1];
  const CT dz = zz - r[2];
  const CT r2 = dx * dx + dy * dy + dz * dz;
  const CT e = kexp2(-r2);
  CT c = r[3] * mj[0];
#pragma unroll
  for (int f = 1; f < FD; f++) c += r[3 + f] * mj[f];
  CT w = c * e;
  if (CUT) {
    // branch-free cutoff: the pair count comes from the scalar unit
    const bool in = r2 <= rc2;
    within_blk = (unsigned)uniform((int)(within_blk + (unsigned)__popcll(__ballot(in))));
    w = in ? w : (CT)0;
  }
  acc.w += w;
  acc.dx += w * dx;
  acc.dy += w * dy;
  acc.dz += w * dz;
}

// The gradient pass's per-lane state: the lane's target (frame
// coordinates, labels), the cutoff and the accumulators.
//
// FP32 (kExpanded) has two forms of the pair, chosen per cluster:
//  * expanded (ex): r^2 = |x|^2 + |z|^2 - 2 x.z with |x|^2 staged beside the
//    source (one add and three fma instead of three subtractions, a product
//    and two fma), accumulating S = sum w x; the item's D = sum w (z - x) is
//    z W - S.  The expansion loses about eps (|x|^2 + |z|^2) of r^2, so it is
//    taken only when the cluster's box lies within kExpandHalf scaled units of
//    its centre (the frame origin): then |x|^2 + |z|^2 stays below ~100.
//  * difference: d = z - x, r^2 = d.d, accumulating D directly (clusters that
//    span more, e.g. long chains of targets at a small length-scale).
// With the cutoff the expanded form is folded: exp2(-r^2) = exp2(-|x|^2)
// exp2(a) with a = 2 x.z - |z|^2 (= |x|^2 - r^2), the source's factor
// exp2(-|x|^2) is multiplied into its labels when it is staged, and the
// cutoff r^2 <= rc2 becomes a >= |x|^2 - rc2, a threshold staged beside the
// source: three fma for the exponent instead of an add and three fma.  A pair
// inside the cutoff has a <= |x|^2 <= ~60 (the box within kExpandHalf of the
// origin, the source within the cutoff of a target), so both factors stay
// normal FP32 numbers; farther pairs (where exp2(a) may overflow against a
// vanishing label factor) are removed by the cutoff's select.
constexpr float kExpandHalf = 3.0f;

template <typename CT, int FD, bool CUT>
struct GradOp {
  static constexpr bool kExpanded = std::is_same<CT, float>::value;
  static constexpr bool kFold = kExpanded && CUT;
  CT zx, zy, zz;
  CT mj[FD];
  CT rc2;
  CT m0, m1, m2, z2;  // expanded form: -2 z, |z|^2; folded: 2 z, -|z|^2
  bool ex;            // the expanded form (wave-uniform)
  Acc<CT> acc;
  // pairs inside the cutoff: a wave-uniform 32-bit count since the last fold
  // (kept in a scalar register), added to the 64-bit total at each fold
  unsigned long long within;
  unsigned int within_blk;
  __device__ __forceinline__ void expand(bool ok) {
    ex = kExpanded && ok;
    const CT two = kFold ? (CT)2 : (CT)-2;
    m0 = two * zx;
    m1 = two * zy;
    m2 = two * zz;
    z2 = zx * zx + zy * zy + zz * zz;
    if (kFold) z2 = -z2;
  }
  // The staged form of a source record s = (x, y, z, labels, extra word) of
  // the expanded form: the extra word is |x|^2, or, folded, the labels are
  // scaled by exp2(-|x|^2) and the extra word is |x|^2 - rc2.
  __device__ __forceinline__ void stage_rec(CT (&s)[3 + FD + 1]) const {
    const CT xx = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
    if (kFold && ex) {
      const CT f = kexp2(-xx);
#pragma unroll
      for (int q = 0; q < FD; q++) s[3 + q] *= f;
      s[3 + FD] = xx - rc2;
    } else {
      s[3 + FD] = xx;
    }
  }
  template <bool E>
  __device__ __forceinline__ void pair_t(const CT* r) {
    if constexpr (E && kFold) {
      const CT a = fma(r[0], m0, fma(r[1], m1, fma(r[2], m2, z2)));  // |x|^2 - r^2
      const CT e = kexp2(a);
      CT c = r[3] * mj[0];
#pragma unroll
      for (int f = 1; f < FD; f++) c += r[3 + f] * mj[f];
      CT w = c * e;
      const bool in = a >= r[3 + FD];  // r^2 <= rc2
      within_blk = (unsigned)uniform((int)(within_blk + (unsigned)__popcll(__ballot(in))));
      w = in ? w : (CT)0;
      acc.w += w;
      acc.dx += w * r[0];
      acc.dy += w * r[1];
      acc.dz += w * r[2];
    } else if constexpr (E) {
      const CT r2 = fma(r[0], m0, fma(r[1], m1, fma(r[2], m2, r[3 + FD] + z2)));
      const CT e = kexp2(-r2);
      CT c = r[3] * mj[0];
#pragma unroll
      for (int f = 1; f < FD; f++) c += r[3 + f] * mj[f];
      CT w = c * e;
      if (CUT) {
        const bool in = r2 <= rc2;
        within_blk = (unsigned)uniform((int)(within_blk + (unsigned)__popcll(__ballot(in))));
        w = in ? w : (CT)0;
      }
      acc.w += w;
      acc.dx += w * r[0];
      acc.dy += w * r[1];
      acc.dz += w * r[2];
    } else {
      one_pair<CT, FD, CUT>(r, zx, zy, zz, mj, rc2, acc, within_blk);
    }
  }
  __device__ __forceinline__ void pair(const CT* r) {
    if (ex) pair_t<true>(r);
    else pair_t<false>(r);
  }
  __device__ __forceinline__ void fold() {
    acc.fold();
    within += within_blk;
    within_blk = 0u;
  }
};

// Accumulators of the quartic pass: the four coefficient sums.
template <typename CT>
struct Acc4;
template <>
struct Acc4<float> {
  float a[4], s[4], c[4];
  __device__ void init() {
#pragma unroll
    for (int q = 0; q < 4; q++) a[q] = s[q] = c[q] = 0.0f;
  }
  __device__ void fold() {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      Acc<float>::kahan(s[q], c[q], a[q]);
      a[q] = 0.0f;
    }
  }
  __device__ void result(double (&out)[4]) {
    fold();
#pragma unroll
    for (int q = 0; q < 4; q++) out[q] = (double)s[q] - (double)c[q];
  }
};
template <>
struct Acc4<double> {
  double a[4];
  __device__ void init() {
#pragma unroll
    for (int q = 0; q < 4; q++) a[q] = 0.0;
  }
  __device__ void fold() {}
  __device__ void result(double (&out)[4]) {
#pragma unroll
    for (int q = 0; q < 4; q++) out[q] = a[q];
  }
};

// The quartic pass (Sec. VI-B, eq. fourth) in the frame's scaled units
// (d^ = s d with s^2 = 1 / (2 ell^2 ln 2), so that -|d|^2/(2 ell^2) =
// -ln2 |d^|^2).  With dk = z~ - x (scaled) and per target
//   u1 = w x z~ + v, u_{k+1} = w x u_k   (the moving target's derivatives),
//   p1 = 2 ln2 u1^, p2 = -ln2 u2^, p3 = ln2/3 u3^, p4 = -ln2/12 u4^,
//   c2 = -ln2 |u1^|^2, c3 = ln2 <u1^,u2^>, c4 = -ln2 (|u2^|^2/4 + <u1^,u3^>/3),
// the exponent of the kernel along the line is
//   alpha + beta t + gamma t^2 + delta t^3 + eps t^4 + O(t^5),
//   beta = <dk,p1>, gamma = c2 + <dk,p2>, delta = c3 + <dk,p3>, eps = c4 + <dk,p4>,
// and the pair adds w g^k with
//   g1 = beta, g2 = gamma + beta^2/2, g3 = delta + beta gamma + beta^3/6,
//   g4 = eps + beta delta + beta^2 gamma/2 + gamma^2/2 + beta^4/24
//      = eps + beta delta + g2^2/2 - beta^4/12.
// The lane keeps gamma, delta and eps halved (their constants scaled by 1/2,
// exactly) and sums g1, g2/2, g3/2 and g4/2:
//   g2/2 = gamma/2 + beta^2/4,  g3/2 = delta/2 + beta (gamma/2 + beta^2/12),
//   g4/2 = (eps/2 + beta delta/2) + (g2/2)^2 - beta^2 (beta^2/24),
// one multiplication fewer than g4 from g2; the item doubles the last three
// sums (exactly) before its wave sums.
template <typename CT, int FD, bool CUT>
struct QuartOp {
  // Expanded form, as in the gradient pass: with dk = z - x,
  // <dk, p> = <z, p> - <x, p>, so each coefficient is one fma chain on the
  // source position with q = -p and the lane's constant k = c + <z, p>, and
  // r^2 = |x|^2 + |z|^2 - 2 x.z; no difference vector is formed.
  static constexpr bool kExpanded = true;
  // FP32 with the cutoff: the folded exponent of the gradient pass
  static constexpr bool kFold = CUT && std::is_same<CT, float>::value;
  CT zx, zy, zz;
  CT mj[FD];
  CT rc2;
  CT q[4][3];         // expanded: -p_k; difference form: p_k (k >= 2: halved)
  CT k1, k2, k3, k4;  // expanded: c_k + <z, p_k>; difference form: c_k (c_1 = 0; k >= 2: halved)
  CT m0, m1, m2, z2;  // -2 z, |z|^2; folded: 2 z, -|z|^2
  bool ex;            // the expanded form (wave-uniform; as for the gradient pass)
  Acc4<CT> acc;
  template <bool E>
  __device__ __forceinline__ void pair_t(const CT* r) {
    // pos: the source (expanded) or d = z - x (difference form)
    CT pos[3], e;
    bool in = true;
    if constexpr (E && kFold) {
      pos[0] = r[0];
      pos[1] = r[1];
      pos[2] = r[2];
      const CT a = fma(r[0], m0, fma(r[1], m1, fma(r[2], m2, z2)));  // |x|^2 - r^2
      e = kexp2(a);
      in = a >= r[3 + FD];
    } else {
      CT r2;
      if constexpr (E) {
        pos[0] = r[0];
        pos[1] = r[1];
        pos[2] = r[2];
        r2 = fma(r[0], m0, fma(r[1], m1, fma(r[2], m2, r[3 + FD] + z2)));
      } else {
        pos[0] = zx - r[0];
        pos[1] = zy - r[1];
        pos[2] = zz - r[2];
        r2 = pos[0] * pos[0] + pos[1] * pos[1] + pos[2] * pos[2];
      }
      e = kexp2(-r2);
      if (CUT) in = r2 <= rc2;
    }
    CT c = r[3] * mj[0];
#pragma unroll
    for (int f = 1; f < FD; f++) c += r[3 + f] * mj[f];
    CT w = c * e;
    if (CUT) w = in ? w : (CT)0;
    const CT be = fma(pos[0], q[0][0], fma(pos[1], q[0][1], fma(pos[2], q[0][2], k1)));
    const CT gah = fma(pos[0], q[1][0], fma(pos[1], q[1][1], fma(pos[2], q[1][2], k2)));  // gamma / 2
    const CT deh = fma(pos[0], q[2][0], fma(pos[1], q[2][1], fma(pos[2], q[2][2], k3)));  // delta / 2
    const CT eph = fma(pos[0], q[3][0], fma(pos[1], q[3][1], fma(pos[2], q[3][2], k4)));  // eps / 2
    const CT b2 = be * be;
    const CT g2h = fma(b2, (CT)0.25, gah);
    const CT g3h = fma(be, fma(b2, (CT)(1.0 / 12.0), gah), deh);
    const CT g4h = fma(-b2, b2 * (CT)(1.0 / 24.0), fma(g2h, g2h, fma(be, deh, eph)));
    acc.a[0] += w * be;
    acc.a[1] += w * g2h;
    acc.a[2] += w * g3h;
    acc.a[3] += w * g4h;
  }
  __device__ __forceinline__ void pair(const CT* r) {
    if (ex) pair_t<true>(r);
    else pair_t<false>(r);
  }
  __device__ __forceinline__ void fold() { acc.fold(); }
  // the staged source record, as for the gradient pass
  __device__ __forceinline__ void stage_rec(CT (&s)[3 + FD + 1]) const {
    const CT xx = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
    if (kFold && ex) {
      const CT f = kexp2(-xx);
#pragma unroll
      for (int q = 0; q < FD; q++) s[3 + q] *= f;
      s[3 + FD] = xx - rc2;
    } else {
      s[3 + FD] = xx;
    }
  }
  // per-target vectors from the direction (w, v) and the target's position
  // zt (m), in FP64, and the lane's frame position (zx, zy, zz, scaled);
  // lanes past the cluster get zero (their pairs have w = 0 and finite g)
  __device__ void setup(const double* __restrict__ xi, const double (&zt)[3], double s, bool valid, bool ok) {
    ex = ok;
    const double w0 = xi[0], w1 = xi[1], w2 = xi[2];
    double u[4][3];
    u[0][0] = w1 * zt[2] - w2 * zt[1] + xi[3];
    u[0][1] = w2 * zt[0] - w0 * zt[2] + xi[4];
    u[0][2] = w0 * zt[1] - w1 * zt[0] + xi[5];
    for (int n = 1; n < 4; n++) {
      u[n][0] = w1 * u[n - 1][2] - w2 * u[n - 1][1];
      u[n][1] = w2 * u[n - 1][0] - w0 * u[n - 1][2];
      u[n][2] = w0 * u[n - 1][1] - w1 * u[n - 1][0];
    }
    for (int n = 0; n < 4; n++)
      for (int a = 0; a < 3; a++) u[n][a] = valid ? u[n][a] * s : 0.0;
    const double ln2 = 0.69314718055994530942;
    const double f[4] = {2.0 * ln2, -ln2, ln2 / 3.0, -ln2 / 12.0};
    double pk[4][3];
    for (int n = 0; n < 4; n++)
      for (int a = 0; a < 3; a++) pk[n][a] = (n > 0 ? 0.5 : 1.0) * f[n] * u[n][a];  // gamma, delta, eps halved
    auto dot = [&](int i, int j) { return u[i][0] * u[j][0] + u[i][1] * u[j][1] + u[i][2] * u[j][2]; };
    const double cc[4] = {0.0, -0.5 * ln2 * dot(0, 0), 0.5 * ln2 * dot(0, 1),
                          -0.5 * ln2 * (0.25 * dot(1, 1) + dot(0, 2) / 3.0)};
    const double z[3] = {(double)zx, (double)zy, (double)zz};
    double kk[4];
    for (int n = 0; n < 4; n++) {
      kk[n] = ex ? cc[n] + z[0] * pk[n][0] + z[1] * pk[n][1] + z[2] * pk[n][2] : cc[n];
      for (int a = 0; a < 3; a++) q[n][a] = (CT)(ex ? -pk[n][a] : pk[n][a]);
    }
    k1 = (CT)kk[0];
    k2 = (CT)kk[1];
    k3 = (CT)kk[2];
    k4 = (CT)kk[3];
    const CT two = kFold ? (CT)2 : (CT)-2;
    m0 = two * zx;
    m1 = two * zy;
    m2 = two * zz;
    z2 = zx * zx + zy * zy + zz * zz;
    if (kFold) z2 = -z2;
    acc.init();
  }
};

// All sources of one cell segment [a, b) of cell (cx, cy, cz) against the
// lane's target, the records moved into the cluster frame as the staging
// does (FP64 offset, one rounding).  The overflow path, when a cluster's
// cell list does not fit.
template <typename CT, int FD, typename Op>
__device__ __forceinline__ void cell_segment(cptr<CT> xr, int xs, int a, int b, int cx, int cy, int cz,
                                             const ClusInfo& ci, Op& op) {
  constexpr int NR = 3 + FD;
  constexpr int NX = NR + (Op::kExpanded ? 1 : 0);
  const double off[3] = {ci.base[0] + cx * ci.hs, ci.base[1] + cy * ci.hs, ci.base[2] + cz * ci.hs};
  for (int b0 = a; b0 < b; b0 += kBlock) {
    const int b1 = min(b0 + kBlock, b);
    for (int i = b0; i < b1; i++) {
      CT rec[NX];
#pragma unroll
      for (int q = 0; q < NR; q++) rec[q] = xr[(size_t)i * xs + q];
#pragma unroll
      for (int q = 0; q < 3; q++) rec[q] = (CT)((double)rec[q] + off[q]);
      if constexpr (Op::kExpanded) op.stage_rec(rec);
      op.pair(rec);
    }
    op.fold();
  }
}

// Can a target within the cluster sphere (centre cc, squared reach
// reach2 = (radius + cutoff reach)^2) have a source in cell (ix, iy, iz)?
__device__ __forceinline__ bool cell_reachable(const GridInfo& g, int ix, int iy, int iz, const double (&cc)[3],
                                               double reach2) {
  if (!g.cutoff) return true;
  const double lo[3] = {g.ox + ix * g.h, g.oy + iy * g.h, g.oz + iz * g.h};
  double d2 = 0.0;
  for (int a = 0; a < 3; a++) {
    const double d = fmax(fmax(lo[a] - cc[a], cc[a] - (lo[a] + g.h)), 0.0);
    d2 += d * d;
  }
  return d2 <= reach2;
}

// SE(3) exponential of the twist (w^, u) (eq. step with t = 1), composed on
// the left of the pose: T <- Exp(w, u) T.  1 - cos th is taken as 2 sin^2(th/2);
// below th = 1e-3 the coefficients use their Taylor series through th^6.
__device__ void left_compose_exp(double T[12], const double w[3], const double u[3]) {
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double th = sqrt(th2);
  double A, B, C;
  if (th < 1e-3) {
    A = 1.0 - th2 * (1.0 / 6.0) + th2 * th2 * (1.0 / 120.0) - th2 * th2 * th2 * (1.0 / 5040.0);
    B = 0.5 - th2 * (1.0 / 24.0) + th2 * th2 * (1.0 / 720.0) - th2 * th2 * th2 * (1.0 / 40320.0);
    C = 1.0 / 6.0 - th2 * (1.0 / 120.0) + th2 * th2 * (1.0 / 5040.0) - th2 * th2 * th2 * (1.0 / 362880.0);
  } else {
    double sn, cs, shalf, chalf;
    sincos(th, &sn, &cs);
    sincos(0.5 * th, &shalf, &chalf);
    A = sn / th;
    B = 2.0 * shalf * shalf / th2;
    C = (th - sn) / (th2 * th);
  }
  // K = w^, K2 = w^ w^ = w w^T - th2 I
  const double K[3][3] = {{0.0, -w[2], w[1]}, {w[2], 0.0, -w[0]}, {-w[1], w[0], 0.0}};
  double R[3][3], V[3][3];
  for (int r = 0; r < 3; r++)
    for (int c = 0; c < 3; c++) {
      const double k2 = w[r] * w[c] - (r == c ? th2 : 0.0);
      const double I = (r == c) ? 1.0 : 0.0;
      R[r][c] = I + A * K[r][c] + B * k2;
      V[r][c] = I + B * K[r][c] + C * k2;
    }
  double t[3];
  for (int r = 0; r < 3; r++) t[r] = V[r][0] * u[0] + V[r][1] * u[1] + V[r][2] * u[2];
  double out[12];
  for (int r = 0; r < 3; r++) {
    for (int c = 0; c < 4; c++) {
      double s = R[r][0] * T[c] + R[r][1] * T[4 + c] + R[r][2] * T[8 + c];
      if (c == 3) s += t[r];
      out[4 * r + c] = s;
    }
  }
  for (int q = 0; q < 12; q++) T[q] = out[q];
}

// ---------------------------------------------------------------------------
// iteration kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_request(const int* __restrict__ clus_end, int nreq, int item) {
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (item < clus_end[mid]) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// XCD-aware block order: consecutive logical blocks share an XCD (L2); the
// hardware places block b on XCD b mod 8.
__device__ __forceinline__ int logical_block() {
  const int nb = gridDim.x;
  const int full = (nb / 8) * 8;
  const int b = blockIdx.x;
  return (b < full) ? (b % 8) * (full / 8) + b / 8 : b;
}

// The cluster's targets: FP64 transformed position and labels.
template <typename CT, int FD>
__device__ __forceinline__ void load_targets(const ReqStatic& R, const double* __restrict__ T, int s0, bool valid,
                                             double (&zt)[3], CT (&mj)[FD]) {
  const int j = s0 + (valid ? lane_id() : 0);
  const float* zr = R.zrec + (size_t)j * R.zs;
  const double z0 = zr[0], z1 = zr[1], z2 = zr[2];
#pragma unroll
  for (int f = 0; f < FD; f++) mj[f] = (CT)zr[3 + f];
  for (int a = 0; a < 3; a++) zt[a] = T[4 * a] * z0 + T[4 * a + 1] * z1 + T[4 * a + 2] * z2 + T[4 * a + 3];
}

// Candidate cell box of the cluster and its bounding sphere, from the
// cluster frame: box [O + blo / sq, O + bhi / sq] (the origin O is the box
// centre) and sphere radius rho = max |z~ - O|.
__device__ __forceinline__ CandBox cand_box_frame(const GridInfo& g, const double (&O)[3], const double (&blo)[3],
                                                  const double (&bhi)[3], double rho) {
  CandBox B;
  int lo[3], hi[3];
  B.pad = 0;
  B.cc[0] = O[0];
  B.cc[1] = O[1];
  B.cc[2] = O[2];
  B.reach2 = INFINITY;
  if (g.cutoff) {
    const double o[3] = {g.ox, g.oy, g.oz};
    const int dim[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; a++) {
      const double bmin = O[a] + blo[a] / g.sq;
      const double bmax = O[a] + bhi[a] / g.sq;
      const double fl = floor((bmin - g.reach - o[a]) / g.h);
      const double fh = floor((bmax + g.reach - o[a]) / g.h);
      lo[a] = (int)fmin(fmax(fl, 0.0), (double)dim[a]);
      hi[a] = (int)fmax(fmin(fh, (double)(dim[a] - 1)), -1.0);
    }
    B.reach2 = (rho + g.reach) * (rho + g.reach);
  } else {
    lo[0] = lo[1] = lo[2] = 0;
    hi[0] = g.nx - 1;
    hi[1] = g.ny - 1;
    hi[2] = g.nz - 1;
  }
  B.rx = uniform(max(hi[0] - lo[0] + 1, 0));
  B.ry = uniform(max(hi[1] - lo[1] + 1, 0));
  B.rz = uniform(max(hi[2] - lo[2] + 1, 0));
  B.ncand = B.rx * B.ry * B.rz;
  B.lo0 = uniform(lo[0]);
  B.lo1 = uniform(lo[1]);
  B.lo2 = uniform(lo[2]);
  return B;
}

// candidate cell t of the box: its key, first source and count (0 if the
// cell is empty or out of reach of the cluster sphere)
__device__ __forceinline__ void cand_cell(const GridInfo& g, const CandBox& B, const int* __restrict__ cs, int t,
                                          int& key, int& first, int& cnt, int* packed = nullptr) {
  key = 0;
  first = 0;
  cnt = 0;
  if (t < B.ncand) {
    const int ix = t % B.rx, iy = (t / B.rx) % B.ry, iz = t / (B.rx * B.ry);
    key = ((B.lo2 + iz) * g.ny + (B.lo1 + iy)) * g.nx + (B.lo0 + ix);
    if (packed) *packed = (B.lo0 + ix) | ((B.lo1 + iy) << 11) | ((B.lo2 + iz) << 22);
    if (cell_reachable(g, B.lo0 + ix, B.lo1 + iy, B.lo2 + iz, B.cc, B.reach2)) {
      first = cs[key];
      cnt = cs[key + 1] - first;
    }
  }
}

// Kernel A: per target cluster (one wavefront each).
//  * The cluster frame: origin O (the centre of the targets' box, FP64), the targets
//    relative to O in scaled units (one rounding to the pair type) with their
//    labels, their bounding box, and the source-grid offsets in the same
//    frame, so that a work item needs no FP64 transform and no dependent
//    look-ups before its first pair.
//  * The compacted list of reachable non-empty source cells in box order, the
//    candidate count, and the cut into work items of at least chunk_min
//    sources (at most chunks_max per cluster) with the list entry that holds
//    each item's first candidate.  The cells of a round (up to 16 per lane,
//    lane-major, so that the list keeps box order) are looked up together.
//  * The items are appended to the launch's work list, one atomic per
//    workgroup; their order there varies from run to run and results do not
//    depend on it (every item has its own output row).
constexpr int kPrepCells = 16;  // candidate cells per lane and round
template <typename CT>
__device__ __forceinline__ void write_frame(const ReqStatic& R, int c, int s0, int cn, const double (&zt)[3],
                                            const GridInfo& g, const double (&O)[3]) {
  const int l = lane_id();
  const bool valid = l < cn;
  const int fd = R.fd;
  CT* blk = (CT*)R.tblk + (size_t)c * (3 + fd) * kWave;
  const CT far = (CT)1e30;
#pragma unroll
  for (int a = 0; a < 3; a++) blk[a * kWave + l] = valid ? (CT)((zt[a] - O[a]) * g.sq) : far;
  const float* zr = R.zrec + (size_t)(s0 + (valid ? l : 0)) * R.zs;
  for (int f = 0; f < fd; f++) blk[(3 + f) * kWave + l] = valid ? (CT)zr[3 + f] : (CT)0;
}

__global__ __launch_bounds__(256) void k_prepare(const ReqStatic* __restrict__ reqs, const int* __restrict__ clus_end,
                                                 int nreq, int total_clusters, QueueRef Q) {
  __shared__ int wcount[kWavesPerBlock];
  __shared__ unsigned int wbase;
  const int w = threadIdx.x >> 6;
  const int lc = uniform(logical_block() * kWavesPerBlock + w);
  const int l = lane_id();
  int nchunks = 0;
  if (lc < total_clusters) {
    const int r = uniform(find_request(clus_end, nreq, lc));
    const ReqStatic& R = reqs[r];
    ReqState* S = R.state;
    const int stage = uniform(S->stage);
    const int c = lc - (r > 0 ? clus_end[r - 1] : 0);
    // launches cover the largest cluster count over the stages
    if (!uniform(S->done) && c < uniform(S->nclus_s[stage])) {
      const int s0 = uniform(R.clus_start[stage][c]);
      const int cn = uniform(R.clus_count[stage][c]);
      const bool valid = l < cn;
      double zt[3];
      float mdummy[1];
      load_targets<float, 1>(R, S->T, s0, valid, zt, mdummy);
      const GridInfo g = R.grid[stage];
      const int* __restrict__ cs = uniform_ptr(R.cstart[stage]);

      // cluster frame: origin at the centre of the targets' bounding box
      // (found relative to the first target, which lane 0 always holds), so
      // that frame coordinates stay small
      const double O0[3] = {uniform_d(zt[0]), uniform_d(zt[1]), uniform_d(zt[2])};
      double blo[3], bhi[3], O[3];
      for (int a = 0; a < 3; a++) {
        const double zr = valid ? (zt[a] - O0[a]) * g.sq : 0.0;
        blo[a] = wave_min(valid ? zr : INFINITY);
        bhi[a] = wave_max(valid ? zr : -INFINITY);
        const double mid = 0.5 * (blo[a] + bhi[a]);
        O[a] = O0[a] + mid / g.sq;
        blo[a] -= mid;
        bhi[a] -= mid;
      }
      if (R.precision == 1)
        write_frame<double>(R, c, s0, cn, zt, g, O);
      else
        write_frame<float>(R, c, s0, cn, zt, g, O);

      // candidate cells, rounds of 64 x kPrepCells in box order (cell
      // t = round base + q * 64 + lane; slots past the box are skipped)
      double rho2 = 0.0;
      for (int a = 0; a < 3; a++) rho2 += valid ? (zt[a] - O[a]) * (zt[a] - O[a]) : 0.0;
      const CandBox B = cand_box_frame(g, O, blo, bhi, sqrt(wave_max(rho2)));
      CellEntry* list = R.cells + (size_t)c * kCellCap;
      int* centry = R.centry + (size_t)c * R.chunks_max;
      constexpr int PR = kWave * kPrepCells;
      const int rounds = (B.ncand + PR - 1) / PR;
      int ccnt[kPrepCells], cfirst[kPrepCells], cpack[kPrepCells];
      auto load_round = [&](int rd) {
#pragma unroll
        for (int q = 0; q < kPrepCells; q++) {
          int key;
          cpack[q] = 0;
          cfirst[q] = 0;
          ccnt[q] = 0;
          if (rd * PR + q * kWave < B.ncand)  // wave-uniform
            cand_cell(g, B, cs, rd * PR + q * kWave + l, key, cfirst[q], ccnt[q], &cpack[q]);
        }
      };
      // pass 1: the candidate count fixes the chunk size
      int total = 0;
      for (int rd = 0; rd < rounds; rd++) {
        load_round(rd);
        int lt = 0;
#pragma unroll
        for (int q = 0; q < kPrepCells; q++) lt += ccnt[q];
        total += wave_sum_int(lt);
      }
      int chunk;
      if (R.mode == kModeEvalTargets) {
        // per-target outputs need all sources of a target in one wavefront
        chunk = total > 0 ? total : 1;
        nchunks = 1;
      } else {
        chunk = (int)(((long long)total + R.chunks_max - 1) / R.chunks_max);
        chunk = chunk < R.chunk_min ? R.chunk_min : chunk;
        nchunks = (int)(((long long)total + chunk - 1) / chunk);
        nchunks = nchunks < 1 ? 1 : nchunks;
      }
      // pass 2: list entries and the entry of each chunk's first candidate
      // (the cells of a single round are still in registers)
      int nl = 0, pos0 = 0;
      for (int rd = 0; rd < rounds; rd++) {
        if (rounds > 1) load_round(rd);
#pragma unroll
        for (int q = 0; q < kPrepCells; q++) {
          if (rd * PR + q * kWave >= B.ncand) break;  // wave-uniform
          const int cnt = ccnt[q];
          const unsigned long long ne = __ballot(cnt > 0);
          const int idx = nl + __popcll(ne & ((1ull << l) - 1ull));
          const int incl = wave_incl_scan(cnt);
          const int pos = pos0 + incl - cnt;
          if (cnt > 0) {
            if (idx < kCellCap) {
              CellEntry e;
              e.cell = cpack[q];
              e.first = cfirst[q];
              e.count = cnt;
              e.end = pos + cnt;
              list[idx] = e;
            }
            // chunks whose first candidate falls in [pos, pos + count)
            for (int kq = (pos + chunk - 1) / chunk; kq < nchunks && (long long)kq * chunk < pos + cnt; kq++)
              centry[kq] = idx < kCellCap ? idx : kCellCap - 1;
          }
          pos0 += lane_value(incl, kWave - 1);
          nl += __popcll(ne);
        }
      }
      // the frame and the counts (all lanes store the same values)
      ClusInfo* ci = R.cinfo + c;
      for (int a = 0; a < 3; a++) {
        ci->O[a] = O[a];
        ci->blo[a] = (float)blo[a];
        ci->bhi[a] = (float)bhi[a];
      }
      ci->base[0] = (g.ox - O[0]) * g.sq;
      ci->base[1] = (g.oy - O[1]) * g.sq;
      ci->base[2] = (g.oz - O[2]) * g.sq;
      ci->hs = g.h * g.sq;
      ci->isq = 1.0 / g.sq;
      ci->xrec = R.xrec[stage];
      ci->total = total;
      ci->ncells = nl;
      ci->overflow = nl > kCellCap ? 1 : 0;
      ci->nchunks = nchunks;
      ci->chunk = chunk;
      ci->s0 = s0;
      ci->cn = cn;
      ci->stage = stage;
      ci->box = B;
    }
  }
  if (l == 0) wcount[w] = nchunks;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int ww = 0; ww < kWavesPerBlock; ww++) t += wcount[ww];
    wbase = t > 0 ? atomicAdd(&Q.q->nitems, (unsigned)t) : 0u;
  }
  __syncthreads();
  if (nchunks > 0) {
    unsigned int base = wbase;
    for (int ww = 0; ww < w; ww++) base += (unsigned)wcount[ww];
    for (int q = l; q < nchunks; q += kWave) {
      const unsigned int it = base + (unsigned)q;
      if (it < Q.cap) Q.items[it] = ((unsigned)lc << kItemShift) | (unsigned)q;
    }
  }
}

template <typename CT, int FD, typename Op>
__device__ __forceinline__ void run_cell(const GridInfo& g, cptr<CT> xr, int xs, int key, int a, int b,
                                         const ClusInfo& ci, Op& op) {
  const int cx = key % g.nx, cy = (key / g.nx) % g.ny, cz = key / (g.nx * g.ny);
  cell_segment<CT, FD, Op>(xr, xs, a, b, cx, cy, cz, ci, op);
}

// F, omega, v from the request's summed terms.
__device__ void gradient_from_sums(const ReqStatic& R, ReqState* __restrict__ S, const double (&acc)[kSlot],
                                   double (&g)[7]) {
  const double ell = R.stage_ell[S->stage];
  const double il2 = 1.0 / (ell * ell);
  g[0] = R.s2f * acc[0];
  for (int a = 0; a < 3; a++) {
    g[1 + a] = R.s2f * acc[1 + a] * il2 / S->a2;
    g[4 + a] = R.s2f * acc[4 + a] * il2 / R.b2;
  }
  for (int q = 0; q < 7; q++) S->g[q] = g[q];
  S->pairs_within += (unsigned long long)acc[7];
  S->pairs_examined += (unsigned long long)acc[8];
}

// The gradient's components in the subgroup the mask selects (the others
// dropped: an orthogonal projection under the diagonal metric a^2, b^2).
__device__ __forceinline__ void masked_gradient(const ReqStatic& R, const double* g, double (&gm)[6]) {
  for (int q = 0; q < 6; q++) gm[q] = ((R.dof_mask >> q) & 1) ? g[1 + q] : 0.0;
}

// <p, q> in the metric: a^2 p_w . q_w + b^2 p_v . q_v
__device__ __forceinline__ double metric_dot(const ReqStatic& R, const ReqState* S, const double* p, const double* q) {
  return S->a2 * (p[0] * q[0] + p[1] * q[1] + p[2] * q[2]) + R.b2 * (p[3] * q[3] + p[4] * q[4] + p[5] * q[5]);
}

// The exponential-map step h <- h exp(tau d) along direction d = (omega, v)
// (the gradient, or a conjugate direction; T <- Exp(-tau d) T), the trace
// row, the stopping test and the stage schedule.
__device__ void take_step(const ReqStatic& R, ReqState* __restrict__ S, double tau, double pairs, const double (&d)[6]) {
  const int stage = S->stage;
  const double ell = R.stage_ell[stage];
  const double* g = S->g;
  S->tau = tau;
  double w[3], u[3], gm[6];
  masked_gradient(R, g, gm);
  for (int a = 0; a < 3; a++) {
    w[a] = -tau * d[a];
    u[a] = -tau * d[3 + a];
  }
  double T[12];
  for (int q = 0; q < 12; q++) T[q] = S->T[q];
  left_compose_exp(T, w, u);
  for (int q = 0; q < 12; q++) S->T[q] = T[q];
  const int k = S->iter;
  if (R.trace) {
    double* tr = R.trace + (size_t)k * kTraceCols;
    for (int q = 0; q < 7; q++) tr[q] = g[q];
    tr[7] = tau;
    tr[8] = ell;
    tr[9] = pairs;
    for (int q = 0; q < 12; q++) tr[10 + q] = T[q];
    tr[22] = 0.0;
    tr[23] = 0.0;
    tr[24] = 0.0;
    tr[25] = 1.0;
  }
  double sq = 0.0, gq = 0.0;
  for (int a = 0; a < 3; a++) {
    sq += w[a] * w[a] + u[a] * u[a];
    gq += gm[a] * gm[a] + gm[3 + a] * gm[3 + a];
  }
  const int kn = k + 1;
  S->iter = kn;
  if (stage == R.n_stages - 1 && (sqrt(sq) < R.tol || sqrt(gq) < R.grad_tol)) {
    S->converged = 1;
    S->done = 1;
  } else if (kn >= R.max_iters) {
    S->done = 1;
  }
  // stage schedule: a stage lasts stage_len iterations, or ends early once
  // the applied twist falls below stage_tol
  if (stage < R.n_stages - 1 && (kn - S->stage_start >= R.stage_len[stage] || sqrt(sq) < R.stage_tol)) {
    S->stage = stage + 1;
    S->stage_start = kn;
  }
}

// The step kernel's work for one request (one thread), by phase:
//  kPhaseFixed     F, omega, v, then the step tau = eta ell^2 / F;
//  kPhaseGradient  F, omega, v only; the direction of the quartic pass is the
//                  gradient (register mode) or the caller's (coefficient mode);
//  kPhaseQuartic   the quartic model's coefficients from the second pass's
//                  sums, then the step at its maximiser (tau = eta ell^2 / F
//                  when the model has no maximum on t > 0).
// The direction of the second pass (S->xi) is the gradient in the mask
// (quartic rule) or the conjugate direction
//   d = g + beta d_prev,  beta = max(0, <g, g - g_prev> / <g_prev, g_prev>)
// (Polak-Ribiere, inner products in the metric), restarted from d = g at the
// first iteration of every length-scale stage, every kCgRestart steps, and
// whenever d is not an ascent direction (<g, d> <= 0).
__device__ void finish_request(const ReqStatic& R, ReqState* __restrict__ S, const double (&acc)[kSlot], int phase) {
  if (phase == kPhaseQuartic) {
    S->A[0] = S->g[0];
    for (int q = 0; q < 4; q++) S->A[1 + q] = R.s2f * acc[q];
    if (R.mode != kModeRegister) {
      S->done = 1;
      return;
    }
    // Along d, A1 = G'(0) = <grad F, d> = a^2 omega . d_w + b^2 v . d_v over
    // the same pairs.  Taken from this identity in FP64: near convergence
    // the terms of the summed A1 cancel to a small remainder that the FP32
    // pair terms resolve only to their rounding, and the step is about
    // -A1 / (2 A2).
    double d[6], gm[6];
    for (int q = 0; q < 6; q++) d[q] = S->xi[q];
    masked_gradient(R, S->g, gm);
    S->A[1] = metric_dot(R, S, gm, d);
    const double ell = R.stage_ell[S->stage];
    double tau = R.eta * ell * ell / S->g[0];
    // The model is trusted while the targets move less than kTrustLengths
    // length-scales: a target z~ moves at speed |d_w x z~ + d_v| along the
    // line, at most |d_w| rho + |d_v| for |z~| <= rho; with rho = zrms + |t|
    // (zrms the targets' root mean square norm) this bounds the typical
    // target's speed.
    const double* Tm = S->T;
    const double rho = S->zrad + sqrt(Tm[3] * Tm[3] + Tm[7] * Tm[7] + Tm[11] * Tm[11]);
    const double speed = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) * rho +
                         sqrt(d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
    const double tmax = speed > 0.0 ? kTrustLengths * ell / speed : INFINITY;
    double t;
    if (quartic_argmax(S->A, &t, tmax)) tau = t;
    take_step(R, S, tau, (double)S->last_pairs, d);
    return;
  }
  double g[7];
  gradient_from_sums(R, S, acc, g);
  if (R.mode == kModeQuartic) {
    return;  // the caller's direction is already in S->xi
  }
  if (R.mode != kModeRegister) {
    S->done = 1;
    return;
  }
  if (!(g[0] > 1e-300)) {
    S->status = -4;  // no pairs in range
    S->done = 1;
    return;
  }
  double gm[6];
  masked_gradient(R, g, gm);
  if (phase == kPhaseGradient) {
    double d[6];
    for (int q = 0; q < 6; q++) d[q] = gm[q];
    if (R.step_rule == kStepConjugate) {
      const int stage = S->stage;
      bool fresh = S->cg_n <= 0 || S->cg_n >= kCgRestart || S->cg_stage != stage;
      if (!fresh) {
        double diff[6];
        for (int q = 0; q < 6; q++) diff[q] = gm[q] - S->gprev[q];
        const double den = metric_dot(R, S, S->gprev, S->gprev);
        double beta = den > 0.0 ? metric_dot(R, S, gm, diff) / den : 0.0;
        beta = beta > 0.0 ? beta : 0.0;
        for (int q = 0; q < 6; q++) d[q] = gm[q] + beta * S->xi[q];
        if (!(metric_dot(R, S, gm, d) > 0.0)) fresh = true;
      }
      if (fresh) {
        for (int q = 0; q < 6; q++) d[q] = gm[q];
        S->cg_n = 0;
      }
      S->cg_n += 1;
      S->cg_stage = stage;
      for (int q = 0; q < 6; q++) S->gprev[q] = gm[q];
    }
    for (int q = 0; q < 6; q++) S->xi[q] = d[q];
    S->last_pairs = (unsigned long long)acc[7];
    return;
  }
  const double ell = R.stage_ell[S->stage];
  take_step(R, S, R.eta * ell * ell / g[0], acc[7], gm);
}

// Wave-local LDS ordering between the lanes of one wavefront.  The LDS
// executes the DS instructions of a wavefront in issue order, so a read issued
// after a write sees it; only the compiler must keep LDS accesses on their side
// of this point.  A wavefront-scope fence does that without waiting for the
// wave's outstanding global loads (a workgroup-scope fence would, and would
// stall the prefetch of the next batch).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Floats per staged source record: x, y, z, labels (and |x|^2 for the
// expanded gradient pass), rounded up to whole 16-byte reads.
template <int FD, bool EXP = false>
struct RecStride {
  static constexpr int value = (3 + FD + (EXP ? 1 : 0) + 3) / 4 * 4;
};

__device__ __forceinline__ unsigned long long wave_or(unsigned long long v) {
  unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
  lo |= (unsigned)dpp32<kDppXor1>((int)lo);
  hi |= (unsigned)dpp32<kDppXor1>((int)hi);
  lo |= (unsigned)dpp32<kDppXor2>((int)lo);
  hi |= (unsigned)dpp32<kDppXor2>((int)hi);
  lo |= (unsigned)dpp32<kDppHalfMirror>((int)lo);
  hi |= (unsigned)dpp32<kDppHalfMirror>((int)hi);
  lo |= (unsigned)dpp32<kDppMirror>((int)lo);
  hi |= (unsigned)dpp32<kDppMirror>((int)hi);
  lo = (unsigned)lane_value((int)lo, 0) | (unsigned)lane_value((int)lo, 16) | (unsigned)lane_value((int)lo, 32) |
       (unsigned)lane_value((int)lo, 48);
  hi = (unsigned)lane_value((int)hi, 0) | (unsigned)lane_value((int)hi, 16) | (unsigned)lane_value((int)hi, 32) |
       (unsigned)lane_value((int)hi, 48);
  return ((unsigned long long)hi << 32) | lo;
}

// A batch of up to 64 consecutive candidate positions of a work item, one per
// lane, with the lane's raw source record in flight.
template <typename CT, int FD>
struct Batch {
  int end;  // one past the batch's last position
  bool live;      // this lane's position is inside the batch
  int cell;       // packed cell coordinates of the lane's source
  CT raw[3 + FD];
};

// Candidate sources [lo_s, hi_s) of the cluster's list, 64 at a time (one per
// lane), software-pipelined: the records of the next batch are requested
// before the current one is culled, staged and paired; the two batches
// alternate between two register sets, so no copy waits for a load in
// flight.  Each record is moved to coordinates relative to the cluster origin
// O (FP64 arithmetic, one rounding to CT) and, with the cutoff, kept only if
// it lies within the cutoff of the cluster's bounding box.  Survivors are
// compacted into the wave's LDS area; a full area is paired with every lane's
// target, each source read at a wave-uniform LDS address.  The list window
// (64 cell entries, one per lane) stays in registers; a position's entry is
// found from a bitmask of the entry boundaries inside the batch.  Returns the
// number of sources paired.
template <typename CT, int FD, bool CUT, typename Op>
__device__ __forceinline__ long long pairs_from_list(const ReqStatic& R, const ClusInfo& ci, int c, int k,
                                                     int lo_s, int hi_s, CT rc2, Op& op, cptr<CT> xr,
                                                     int xs, CT* recs) {
  constexpr int RS = RecStride<FD, Op::kExpanded>::value;
  constexpr int NX = 3 + FD + (Op::kExpanded ? 1 : 0);  // floats read per record
  constexpr int NR = (sizeof(CT) == 4) ? kStage32 : kStage64;
  static_assert(NR % kWave == 0 && NR >= kWave, "a staging round holds at least one batch");
  const int l = lane_id();
  const CellEntry* __restrict__ list = uniform_ptr(R.cells + (size_t)c * kCellCap);
  const int nl = uniform(ci.ncells);
  // cluster bounding box in the frame's scaled coordinates; a source farther
  // than the cutoff from it cannot pair with any target (threshold widened by
  // a relative 1e-4 so that no pair the per-pair test accepts is dropped)
  const CT blo[3] = {(CT)ci.blo[0], (CT)ci.blo[1], (CT)ci.blo[2]};
  const CT bhi[3] = {(CT)ci.bhi[0], (CT)ci.bhi[1], (CT)ci.bhi[2]};
  const CT cull2 = rc2 * (CT)1.0001 + (CT)1e-6;
  // offset of cell (0,0,0) from the origin, in scaled units
  const double base[3] = {ci.base[0], ci.base[1], ci.base[2]};
  const double hs = ci.hs;
  const CT* xg0 = (const CT*)xr;

  // entry window: lane k holds entry we0 + k (the entry holding the item's
  // first candidate was found by the prepare kernel)
  int we0 = uniform(R.centry[(size_t)c * R.chunks_max + k]);
  int navail = 0;
  int win_end = 0;  // positions are ints: a cluster's candidates number below 2^31
  CellEntry me;
  // Loads below are issued by every lane (dead lanes read a valid clamped
  // address): a load under a branch would make the compiler's wait counts
  // assume it might not have been issued, and wait for the batch in flight.
  // The window load is consumed by selects (no branch) right away, so no
  // path leaves it in flight.
  static_assert(sizeof(CellEntry) == 4 * sizeof(int), "a cell entry is four ints");
  const __attribute__((address_space(1))) int* glist = (const __attribute__((address_space(1))) int*)list;
  auto load_window = [&]() {
    navail = uniform(min(kWave, nl - we0));
    const bool in = l < navail;
    const int idx = we0 + (in ? l : 0);
    const int e4 = 4 * (idx < nl && idx >= 0 ? idx : 0);
    const int ecell = glist[e4], efirst = glist[e4 + 1], ecount = glist[e4 + 2], eend = glist[e4 + 3];
    me.cell = in ? ecell : 0;
    me.first = in ? efirst : 0;
    me.count = in ? ecount : 0;
    me.end = in ? eend : 0x7fffffff;
    const int last_end = lane_value(me.end, navail > 0 ? navail - 1 : 0);
    win_end = navail > 0 ? last_end : hi_s;
  };
  // request the records of the batch starting at pos
  auto start_batch = [&](int pos, Batch<CT, FD>& B) {
    if (pos >= win_end) {
      we0 += navail;
      load_window();
    }
    int bend = (hi_s - pos < kWave) ? hi_s : pos + kWave;
    if (bend > win_end) bend = win_end;
    B.end = bend;
    B.live = l < bend - pos;
    const int p = pos + (B.live ? l : 0);
    // entries of the window that end at or before pos, and the entry
    // boundaries inside the batch
    const int bk = me.end - pos;  // (me.end >= 0, pos >= 0: no overflow)
    const int eoff = __popcll(__ballot(l < navail && bk <= 0));
    const bool inside = l < navail && bk >= 1 && bk <= kWave - 1;
    int efirst, ecount, eend;
    if (__ballot(inside) == 0ull) {
      // no entry ends inside the batch (the common case with large cells):
      // every lane's entry is eoff, read with scalar lane reads
      int e = eoff < navail - 1 ? eoff : navail - 1;
      e = e < 0 ? 0 : e;
      efirst = lane_value(me.first, e);
      ecount = lane_value(me.count, e);
      eend = lane_value(me.end, e);
      B.cell = lane_value(me.cell, e);
    } else {
      const unsigned long long M = wave_or(inside ? (1ull << bk) : 0ull);
      const unsigned long long upto = (l == kWave - 1) ? ~1ull : ((2ull << l) - 2ull);  // bits 1..l
      int ei = eoff + __popcll(M & upto);
      ei = ei < navail - 1 ? ei : navail - 1;
      ei = ei < 0 ? 0 : ei;
      efirst = __shfl(me.first, ei, kWave);
      ecount = __shfl(me.count, ei, kWave);
      eend = __shfl(me.end, ei, kWave);
      B.cell = __shfl(me.cell, ei, kWave);
    }
    const int src = B.live ? efirst + (p - (eend - ecount)) : 0;
    const CT* xg = xg0 + (size_t)src * xs;
#pragma unroll
    for (int q = 0; q < 3 + FD; q++) B.raw[q] = xg[q];
  };

  long long paired = 0;
  int count = 0;  // staged survivors
  // the pairing of a full staging area, one copy of the loop per form of
  // the pair (the form is fixed per item)
  auto pair_all = [&](auto form) {
    constexpr bool E = decltype(form)::value;
    constexpr int U = 4;
    for (int b0 = 0; b0 < count; b0 += kBlock) {
      const int b1 = min(b0 + kBlock, count);
      int i = b0;
      for (; i + U <= b1; i += U) {
        CT r4[U][NX];
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
          for (int q = 0; q < NX; q++) r4[u][q] = recs[(i + u) * RS + q];
#pragma unroll
        for (int u = 0; u < U; u++) op.template pair_t<E>(r4[u]);
      }
      for (; i < b1; i++) {
        CT r1[NX];
#pragma unroll
        for (int q = 0; q < NX; q++) r1[q] = recs[i * RS + q];
        op.template pair_t<E>(r1);
      }
      op.fold();
    }
  };
  auto flush = [&]() {
    wave_lds_sync();
    if (Op::kExpanded && op.ex)
      pair_all(std::integral_constant<bool, Op::kExpanded>());
    else
      pair_all(std::false_type());
    paired += count;
    count = 0;
    wave_lds_sync();
  };
  // cull batch B, append its survivors to the staging area, pair a full area
  // (or everything, after the last batch)
  // (every lane computes its record, live or not, so that no path skips the
  // use of the batch's loads)
  auto stage = [&](const Batch<CT, FD>& B, bool last) {
    CT rec[3 + FD];
    const int cx = B.cell & 2047, cy = (B.cell >> 11) & 2047, cz = (B.cell >> 22) & 2047;
    rec[0] = (CT)((double)B.raw[0] + (base[0] + cx * hs));
    rec[1] = (CT)((double)B.raw[1] + (base[1] + cy * hs));
    rec[2] = (CT)((double)B.raw[2] + (base[2] + cz * hs));
    // (the first label is passed through an add so that the staged record's
    // first four words are formed here, not moved out of the load's registers
    // at the loop's back edge; x + 0 only turns -0 into +0)
    rec[3] = B.raw[3] + (CT)0;
#pragma unroll
    for (int f = 1; f < FD; f++) rec[3 + f] = B.raw[3 + f];
    bool keep = B.live;
    if (CUT) {
      CT d2 = 0;
#pragma unroll
      for (int a = 0; a < 3; a++) {
        const CT d = fmax(fmax(blo[a] - rec[a], rec[a] - bhi[a]), (CT)0);
        d2 += d * d;
      }
      keep = keep && d2 <= cull2;
    }
    const unsigned long long km = __ballot(keep);
    if (keep) {
      CT* dst = recs + (count + __popcll(km & ((1ull << l) - 1ull))) * RS;
      if constexpr (Op::kExpanded) {
        CT srec[3 + FD + 1];
#pragma unroll
        for (int q = 0; q < 3 + FD; q++) srec[q] = rec[q];
        op.stage_rec(srec);
#pragma unroll
        for (int q = 0; q < 3 + FD + 1; q++) dst[q] = srec[q];
      } else {
#pragma unroll
        for (int q = 0; q < 3 + FD; q++) dst[q] = rec[q];
      }
    }
    count += __popcll(km);
    if (count > NR - kWave || (last && count > 0)) flush();
  };

  load_window();
  if (navail <= 0) return 0;
  // A starts as an empty batch (no loads), so both batches enter the loop in
  // the registers the loop keeps them in.  The next batch is always requested
  // (past the end it is empty: no live lane, loads of record 0), so the loads
  // in flight are the same on every path and the waits before staging count
  // only the older batch.
  Batch<CT, FD> A, B;
  A.end = lo_s;
  A.live = false;
  A.cell = 0;
#pragma unroll
  for (int q = 0; q < 3 + FD; q++) A.raw[q] = (CT)0;
  int pos = lo_s;
  for (;;) {
    const bool moreB = pos < hi_s;
    start_batch(pos, B);
    pos = B.end > pos ? B.end : pos;
    stage(A, !moreB);
    if (!moreB) break;
    const bool moreA = pos < hi_s;
    start_batch(pos, A);
    pos = A.end > pos ? A.end : pos;
    stage(B, !moreA);
    if (!moreA) break;
  }
  return paired;
}

// One work item: candidate sources [k chunk, (k + 1) chunk) of cluster c
// against the cluster's targets (one per lane), in the frame the prepare
// kernel set up.  The item's sums go to its own row: W, the torque and
// translation terms and the pair counts (gradient pass), or the four
// quartic-model sums (QUART).
template <typename CT, int FD, bool CUT, bool QUART>
__device__ __forceinline__ void process_item(const ReqStatic* __restrict__ reqs, const int* __restrict__ clus_end,
                                             int nreq, int lc, int k, CT* recs) {
  const int r = uniform(find_request(clus_end, nreq, lc));
  const ReqStatic& R = reqs[r];
  const int c = lc - (r > 0 ? clus_end[r - 1] : 0);
  const int l = lane_id();
  const ClusInfo& ci = R.cinfo[c];
  const int total = uniform(ci.total);
  const int chunk = uniform(ci.chunk);
  const int cn = uniform(ci.cn);
  const int lo_s = k * chunk;  // k < chunks of the cluster: below total
  const int hi_s = (total - lo_s < chunk) ? total : lo_s + chunk;
  const bool valid = l < cn;
  // targets in the cluster frame, and labels
  const CT* blk = (const CT*)R.tblk + (size_t)c * (3 + FD) * kWave;
  const CT zx = blk[l], zy = blk[kWave + l], zz = blk[2 * kWave + l];
  using Op = typename std::conditional<QUART, QuartOp<CT, FD, CUT>, GradOp<CT, FD, CUT>>::type;
  Op op;
  op.zx = zx;
  op.zy = zy;
  op.zz = zz;
#pragma unroll
  for (int f = 0; f < FD; f++) op.mj[f] = blk[(3 + f) * kWave + l];
  const CT rc2 = (CT)R.grid[0].rc2s;  // the same for every stage
  op.rc2 = rc2;
  const cptr<CT> xr = (cptr<CT>)uniform_ptr(ci.xrec);
  const int xs = uniform(R.xs);
  const double isq = ci.isq;
  const bool overflow = uniform(ci.overflow) != 0;
  // the expanded pair form keeps its precision while the cluster's box stays
  // within kExpandHalf scaled units of the frame origin (its centre)
  bool expand_ok = true;
#pragma unroll
  for (int a = 0; a < 3; a++) expand_ok = expand_ok && fmaxf(-ci.blo[a], ci.bhi[a]) <= kExpandHalf;

  // the target position z~_j (m): the torque's lever, the quartic vectors'
  // base point (FP64 from the pose when the list overflowed)
  double zt[3] = {0.0, 0.0, 0.0};
  if (overflow) {
    CT mdummy[FD];
    load_targets<CT, FD>(R, R.state->T, uniform(ci.s0), valid, zt, mdummy);
  }
  auto lever = [&](double (&p)[3]) {
    p[0] = overflow ? zt[0] : ci.O[0] + (double)zx * isq;
    p[1] = overflow ? zt[1] : ci.O[1] + (double)zy * isq;
    p[2] = overflow ? zt[2] : ci.O[2] + (double)zz * isq;
  };
  if constexpr (QUART) {
    double lv[3];
    lever(lv);
    op.setup(R.state->xi, lv, 1.0 / isq, valid, expand_ok);
  } else {
    op.expand(expand_ok);
    op.acc.init();
    op.within = 0;
    op.within_blk = 0u;
  }
  long long span = 0;
  if (!overflow) {
    if (lo_s < hi_s) span = pairs_from_list<CT, FD, CUT, Op>(R, ci, c, k, lo_s, hi_s, rc2, op, xr, xs, recs);
  } else {
    // the list overflowed: enumerate the candidate box the prepare kernel
    // counted again, in the same order
    const GridInfo g = R.grid[uniform(ci.stage)];
    const int* __restrict__ cs = uniform_ptr(R.cstart[uniform(ci.stage)]);
    const CandBox B = ci.box;
    long long base = 0;
    for (int c0 = 0; c0 < B.ncand && base < hi_s; c0 += kWave) {
      int key, first, cnt;
      cand_cell(g, B, cs, c0 + l, key, first, cnt);
      const int incl = wave_incl_scan(cnt);
      const long long cb = base + incl - cnt, ce = base + incl;
      unsigned long long todo = __ballot(cnt > 0 && ce > lo_s && cb < hi_s);
      while (todo) {
        const int src = __builtin_ctzll(todo);
        todo &= todo - 1ull;
        const int ckey = lane_value(key, src);
        const int cfirst = lane_value(first, src);
        const int ccnt = lane_value(cnt, src);
        const long long cbeg = base + lane_value(incl - cnt, src);
        const int a = cfirst + (int)(lo_s > cbeg ? lo_s - cbeg : 0);
        const int b = cfirst + (int)((hi_s - cbeg) < ccnt ? (hi_s - cbeg) : ccnt);
        run_cell<CT, FD, Op>(g, xr, xs, ckey, a, b, ci, op);
        span += b - a;
      }
      base += lane_value(incl, kWave - 1);
    }
  }
  double* row = R.sslots + ((size_t)c * R.chunks_max + k) * kSlot;
  if constexpr (QUART) {
    double a4[4];
    op.acc.result(a4);
#pragma unroll
    for (int q = 0; q < 4; q++) a4[q] = valid ? (q > 0 ? 2.0 * a4[q] : a4[q]) : 0.0;  // the halved sums
    const double part[kSlot] = {wave_sum(a4[0]), wave_sum(a4[1]), wave_sum(a4[2]), wave_sum(a4[3]), 0.0, 0.0,
                                0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < kSlot; q++) row[q] = part[q];
  } else {
    unsigned long long within = op.within + op.within_blk;
    const unsigned long long examined = (unsigned long long)span * (unsigned long long)cn;
    if (!CUT) within = examined;

    double W, Dx, Dy, Dz;
    op.acc.result(W, Dx, Dy, Dz);
    if (op.ex) {
      // S = sum w x  ->  D = sum w (z - x) = z W - S
      Dx = (double)zx * W - Dx;
      Dy = (double)zy * W - Dy;
      Dz = (double)zz * W - Dz;
    }
    if (!valid) W = Dx = Dy = Dz = 0.0;
    Dx *= isq;
    Dy *= isq;
    Dz *= isq;
    // sum_i w (x_i x z~_j) = z~_j x D_j with D_j = sum_i w (z~_j - x_i)
    double lv[3];
    lever(lv);
    const double ox = lv[1] * Dz - lv[2] * Dy;
    const double oy = lv[2] * Dx - lv[0] * Dz;
    const double oz = lv[0] * Dy - lv[1] * Dx;

    // (wave-uniform values are read outside the lane-dependent branch)
    const int s0 = uniform(ci.s0);
    const double ell_c = R.stage_ell[uniform(ci.stage)];
    if (R.mode == kModeEvalTargets && R.per_target && valid) {
      const double il2 = 1.0 / (ell_c * ell_c);
      const double a2 = R.state->a2;
      double* o = R.per_target + (size_t)R.zorig[s0 + l] * 7;
      o[0] = R.s2f * W;
      o[1] = R.s2f * ox * il2 / a2;
      o[2] = R.s2f * oy * il2 / a2;
      o[3] = R.s2f * oz * il2 / a2;
      o[4] = R.s2f * Dx * il2 / R.b2;
      o[5] = R.s2f * Dy * il2 / R.b2;
      o[6] = R.s2f * Dz * il2 / R.b2;
    }

    const double part[kSlot] = {wave_sum(W),  wave_sum(ox), wave_sum(oy),     wave_sum(oz),    wave_sum(Dx),
                                wave_sum(Dy), wave_sum(Dz), (double)within, (double)examined};
    // every lane holds the same sums: all lanes store them (same address,
    // same value), so the persistent loop has no lane-dependent branch
#pragma unroll
    for (int q = 0; q < kSlot; q++) row[q] = part[q];
  }
}

// Kernel B: persistent workgroups, as many as are resident at once (two per
// compute unit).  Workgroup b takes an equal share of the launch's work items
// (see below); its wavefronts take the items of the share one at a time from
// a counter in LDS, so the compute unit stays busy until its share is done and
// no device-wide atomic is needed (one same-address device atomic per item
// costs more than the items' arithmetic at this granularity).  Results do not
// depend on which wavefront takes an item.  Every wavefront reaches the exit:
// the counter grows by one per take and the share is finite.
template <typename CT>
struct PairWaves {
  // one 16-wave workgroup per CU for FP32 (4 waves per SIMD at <= 128 VGPRs);
  // the FP64 instances need more registers: two waves per SIMD, 8-wave groups
  static constexpr int value = sizeof(CT) == 4 ? kPairBlockWaves : kPairBlockWaves / 2;
};

template <typename CT, int FD, bool CUT, bool QUART>
__global__ __launch_bounds__((PairWaves<CT>::value * kWave), (sizeof(CT) == 4 ? 4 : 2)) void k_pairs(const ReqStatic* __restrict__ reqs,
                                                                  const int* __restrict__ clus_end, int nreq,
                                                                  QueueRef Q) {
  constexpr int RS = RecStride<FD, std::is_same<CT, float>::value || QUART>::value;
  constexpr int NR = (sizeof(CT) == 4) ? kStage32 : kStage64;
  __shared__ __align__(16) CT recs_all[PairWaves<CT>::value][NR * RS];
  __shared__ unsigned int next;
  CT* recs = recs_all[threadIdx.x >> 6];
  const unsigned int nitems = (unsigned)uniform((int)min(Q.q->nitems, Q.cap));
  const unsigned long long G = gridDim.x;
  // Shares: the workgroups of one XCD (the hardware places workgroup b on
  // XCD b mod 8) take a contiguous range of the list, so a cluster's items
  // (adjacent in the list) share that XCD's L2.  The range is cut into blocks
  // of cx items (cx = the XCD's workgroup count); in block t workgroup rk
  // takes position (rk + h(t)) mod cx, h a hash of t: one item per workgroup
  // and block, each item exactly once.  The offset moves from block to block
  // because an item's cost depends on its position in its cluster's candidate
  // list (the first and last chunks hold the cells at the ends of the
  // candidate box, whose sources mostly fail the cull): with a fixed stride a
  // workgroup would keep drawing the same positions of clusters with about
  // cx items, and the shares' costs would not even out.
  const unsigned int b = blockIdx.x, x = b % 8u, rk = b / 8u;
  unsigned long long before = 0;
  for (unsigned int y = 0; y < x; y++) before += (G - y + 7u) / 8u;
  const unsigned int cx = (unsigned)((G - x + 7u) / 8u);
  const unsigned int lo = (unsigned)((unsigned long long)nitems * before / G);
  const unsigned int hi = (unsigned)((unsigned long long)nitems * (before + cx) / G);
  const unsigned int nx = hi - lo;
  const unsigned int nblk = (nx + cx - 1u) / cx;
  if (threadIdx.x == 0) next = 0u;
  __syncthreads();
  // No branch on the lane index may sit in this loop: the compiler may thread
  // the loop's back edge on such a branch, which splits the wavefront so that
  // lanes 1..63 re-enter the body without lane 0 and never see a new ticket.
  // Every lane takes part in the atomic (lane 0 adds one, the others zero)
  // and the ticket is lane 0's result.
  for (;;) {
    const unsigned int mine = atomicAdd(&next, lane_id() == 0 ? 1u : 0u);
    const unsigned int t = (unsigned)uniform((int)mine);
    if (t >= nblk) break;
    const unsigned int pos = t * cx + (rk + (t * 2654435761u) % cx) % cx;
    if (pos >= nx) continue;  // the last block may be partial
    const unsigned int item = uniform((int)Q.items[lo + pos]);
    process_item<CT, FD, CUT, QUART>(reqs, clus_end, nreq, (int)(item >> kItemShift),
                              (int)(item & ((1u << kItemShift) - 1u)), recs);
  }
}

// Kernel C1: per target cluster (one wavefront each), the sum of its work-item
// rows: lane j holds chunk j (zero past the cluster's count), summed by the
// fixed xor butterfly, so the result does not depend on the order in which the
// items ran.  After the iteration's last pass block 0 also resets the work
// list for the next launch (the quartic pass reuses the gradient pass's items).
__global__ __launch_bounds__(256) void k_reduce(const ReqStatic* __restrict__ reqs, const int* __restrict__ clus_end,
                                                int nreq, int total_clusters, QueueRef Q, int reset) {
  if (reset && blockIdx.x == 0 && threadIdx.x == 0) Q.q->nitems = 0u;
  const int lc = uniform(blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6));
  if (lc >= total_clusters) return;
  const int r = uniform(find_request(clus_end, nreq, lc));
  const ReqStatic& R = reqs[r];
  if (uniform(R.state->done)) return;
  const int c = lc - (r > 0 ? clus_end[r - 1] : 0);
  const int l = lane_id();
  // clusters past the current stage's count hold no items: a zero row.
  // Lane l holds chunks l, l + 64, l + 128, l + 192 (those that exist),
  // added in that order.
  const int nch = c < uniform(R.state->nclus_s[uniform(R.state->stage)]) ? uniform(R.cinfo[c].nchunks) : 0;
  const double* rows = R.sslots + (size_t)c * R.chunks_max * kSlot;
  double v[kSlot];
#pragma unroll
  for (int q = 0; q < kSlot; q++) v[q] = 0.0;
  for (int b = 0; b < kChunksCap; b += kWave) {
    if (b >= nch) break;  // wave-uniform
    const bool has = b + l < nch;
    const double* row = rows + (size_t)(has ? b + l : 0) * kSlot;
#pragma unroll
    for (int q = 0; q < kSlot; q++) {
      const double x = row[q];
      v[q] += has ? x : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < kSlot; q++) v[q] = wave_sum(v[q]);
  // every lane holds the sums; all store them (same address, same value)
  double* out = R.csum + (size_t)c * kSlot;
#pragma unroll
  for (int q = 0; q < kSlot; q++) out[q] = v[q];
}

// Kernel C2: one 512-thread block per request.  Thread t sums the cluster rows
// t, t + 512, ... in order; the 512 thread sums are combined by a fixed tree
// (wave butterflies, then waves in order): a deterministic FP64 reduction,
// then the step.
constexpr int kStepThreads = 512;
__global__ __launch_bounds__(kStepThreads) void k_step(const ReqStatic* __restrict__ reqs, int nreq, int phase) {
  const int r = blockIdx.x;
  if (r >= nreq) return;
  const ReqStatic& R = reqs[r];
  ReqState* S = R.state;
  if (S->done) return;  // block-uniform
  constexpr int NW = kStepThreads / kWave;
  __shared__ double wsum[NW][kSlot];
  const int w = threadIdx.x >> 6;
  const int l = lane_id();
  double acc[kSlot];
#pragma unroll
  for (int q = 0; q < kSlot; q++) acc[q] = 0.0;
  const int nrows = R.nclus;
  int i = threadIdx.x;
  for (; i + 3 * kStepThreads < nrows; i += 4 * kStepThreads) {
    double v[4][kSlot];
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
      for (int q = 0; q < kSlot; q++) v[u][q] = R.csum[(size_t)(i + u * kStepThreads) * kSlot + q];
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
      for (int q = 0; q < kSlot; q++) acc[q] += v[u][q];
  }
  for (; i < nrows; i += kStepThreads)
#pragma unroll
    for (int q = 0; q < kSlot; q++) acc[q] += R.csum[(size_t)i * kSlot + q];
#pragma unroll
  for (int q = 0; q < kSlot; q++) acc[q] = wave_sum(acc[q]);
  if (l == 0)
    for (int q = 0; q < kSlot; q++) wsum[w][q] = acc[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[kSlot];
    for (int q = 0; q < kSlot; q++) {
      double t = 0.0;
      for (int ww = 0; ww < NW; ww++) t += wsum[ww][q];
      tot[q] = t;
    }
    finish_request(R, S, tot, phase);
  }
}

// ---------------------------------------------------------------------------
// 7) request state set-up
// ---------------------------------------------------------------------------
__global__ void k_init_state(ReqState* __restrict__ S, const double* __restrict__ T0, const double* __restrict__ xi0,
                             double a2_param) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int q = 0; q < 12; q++) S->T[q] = T0[q];
  for (int q = 0; q < 7; q++) S->g[q] = 0.0;
  for (int q = 0; q < 6; q++) S->xi[q] = xi0 ? xi0[q] : 0.0;
  for (int q = 0; q < 6; q++) S->gprev[q] = 0.0;
  S->cg_n = 0;
  S->cg_stage = 0;
  S->stage_start = 0;
  for (int q = 0; q < 5; q++) S->A[q] = 0.0;
  S->last_pairs = 0ull;
  S->a2 = a2_param;
  S->zrad = 0.0;
  S->tau = 0.0;
  S->pairs_within = 0ull;
  S->pairs_examined = 0ull;
  S->iter = 0;
  S->stage = 0;
  S->done = 0;
  S->status = 0;
  S->converged = 0;
  S->reserved = 0u;
  S->bad_input = 0;
  S->nclus = 0;
  for (int st = 0; st < kMaxStages; st++) S->nclus_s[st] = 0;
}

__global__ __launch_bounds__(256) void k_check_finite(const float* __restrict__ p, long long count,
                                                      ReqState* __restrict__ S) {
  bool bad = false;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    bad |= !isfinite(p[i]);
  if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(&S->bad_input, 1);
}

__global__ void k_setup_final(ReqState* __restrict__ S, const double* __restrict__ xbox,
                              const double* __restrict__ zbox, double a2_param, int n_stages) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (!(a2_param > 0.0)) S->a2 = xbox[6];
  S->zrad = sqrt(zbox[6]);  // root mean square norm of the targets
  int most = 0, least = 0x7fffffff;
  for (int st = 0; st < n_stages; st++) {
    most = max(most, S->nclus_s[st]);
    least = min(least, S->nclus_s[st]);
  }
  S->nclus = most;
  if (S->bad_input || !(S->a2 > 0.0) || !isfinite(S->a2) || least < 1) {
    S->status = -1;  // invalid input
    S->done = 1;
  }
}

// ---------------------------------------------------------------------------
// RGB-D front end (Sec. VII-B, TUM experiment): semi-dense selection of the
// pixels of largest image gradient and their points from the organised depth
// image.  Every floating-point step that decides the selection is fixed in
// FP32 (no contraction), so the kept set is exact:
//   I = ((r + g) + b) / 3;  gu, gv central differences (one-sided at the
//   border);  s = gu*gu + gv*gv;  valid = finite depth in [dmin, dmax];
//   keep the k valid pixels of largest s, ties to the smaller pixel index,
//   in increasing pixel order.
// Selection is a two-level radix select on key = bits(s) + 1 (0: invalid):
// 16-bit histograms find the k-th largest key t; the pixels with key > t and
// the first (k - #{key > t}) pixels with key == t in pixel order are kept.
// ---------------------------------------------------------------------------
constexpr int kFeBins = 1 << 16;

__global__ __launch_bounds__(256) void k_fe_intensity(const float* __restrict__ rgb, long long P,
                                                      float* __restrict__ I, FeCtl* __restrict__ ctl) {
  bool bad = false;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += (long long)gridDim.x * blockDim.x) {
    const float r = rgb[3 * p], g = rgb[3 * p + 1], b = rgb[3 * p + 2];
    bad |= !(isfinite(r) && isfinite(g) && isfinite(b));
    I[p] = ((r + g) + b) / 3.0f;
  }
  if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(&ctl->bad, 1);
}

// gu, gv at pixel (u, v), the border rules of the definition
__device__ __forceinline__ void fe_grad(const float* __restrict__ I, int W, int H, int u, int v, float& gu, float& gv) {
  const float* row = I + (size_t)v * W;
  if (W < 2) gu = 0.0f;
  else if (u == 0) gu = row[1] - row[0];
  else if (u == W - 1) gu = row[W - 1] - row[W - 2];
  else gu = (row[u + 1] - row[u - 1]) / 2.0f;
  if (H < 2) gv = 0.0f;
  else if (v == 0) gv = I[(size_t)W + u] - I[u];
  else if (v == H - 1) gv = I[(size_t)(H - 1) * W + u] - I[(size_t)(H - 2) * W + u];
  else gv = (I[(size_t)(v + 1) * W + u] - I[(size_t)(v - 1) * W + u]) / 2.0f;
}

__device__ __forceinline__ float fe_score(float gu, float gv) {
#pragma clang fp contract(off)
  const float a = gu * gu;
  const float b = gv * gv;
  return a + b;
}

__global__ __launch_bounds__(256) void k_fe_score(const float* __restrict__ I, const float* __restrict__ depth, int W,
                                                  int H, float dmin, float dmax, unsigned* __restrict__ key,
                                                  unsigned* __restrict__ hist) {
  const long long P = (long long)W * H;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += (long long)gridDim.x * blockDim.x) {
    const int v = (int)(p / W), u = (int)(p - (long long)v * W);
    float gu, gv;
    fe_grad(I, W, H, u, v, gu, gv);
    const float s = fe_score(gu, gv);
    const float d = depth[p];
    const bool valid = isfinite(d) && d >= dmin && d <= dmax;
    const unsigned kk = valid ? __float_as_uint(s) + 1u : 0u;  // s >= 0 and finite: bits are monotone
    key[p] = kk;
    if (kk) atomicAdd(&hist[kk >> 16], 1u);
  }
}

// One 1024-thread block: the high-16-bit bin holding the k-th largest key
// (thread t holds bins 64t .. 64t + 63, scanned from the top), and the number
// of keys in the bins above it.  When at most k pixels are valid all are kept.
__global__ __launch_bounds__(1024) void k_fe_find(const unsigned* __restrict__ hist, int k, FeCtl* __restrict__ ctl) {
  constexpr int per = kFeBins / 1024;
  __shared__ int sh[33];
  const int t = threadIdx.x;
  const int rt = 1023 - t;  // reversed order: thread 0 holds the top bins
  int sum = 0;
  for (int q = 0; q < per; q++) sum += (int)hist[rt * per + q];
  int total;
  int above = block_excl_scan(sum, sh, total);  // keys in the bins above this thread's range
  if (t == 0) {
    ctl->valid = total;
    ctl->all = total <= k ? 1 : 0;
  }
  if (total <= k) return;  // block-uniform
  if (above < k && above + sum >= k) {
    for (int q = per - 1; q >= 0; q--) {
      const int b = rt * per + q;
      const int c = (int)hist[b];
      if (above + c >= k) {
        ctl->hi = b;
        ctl->above = above;
        break;
      }
      above += c;
    }
  }
}

// level 1 of the search, skipped when every valid pixel is kept
__global__ __launch_bounds__(1024) void k_fe_find_lo_gate(const unsigned* __restrict__ hist, int k,
                                                          FeCtl* __restrict__ ctl);

__global__ __launch_bounds__(256) void k_fe_hist_lo(const unsigned* __restrict__ key, long long P,
                                                    const FeCtl* __restrict__ ctl, unsigned* __restrict__ hist) {
  if (ctl->all) return;
  const unsigned hi = (unsigned)ctl->hi;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += (long long)gridDim.x * blockDim.x) {
    const unsigned kk = key[p];
    if (kk && (kk >> 16) == hi) atomicAdd(&hist[kk & 0xFFFFu], 1u);
  }
}

__global__ __launch_bounds__(1024) void k_fe_find_lo_gate(const unsigned* __restrict__ hist, int k,
                                                          FeCtl* __restrict__ ctl) {
  if (ctl->all) return;  // block-uniform
  constexpr int per = kFeBins / 1024;
  __shared__ int sh[33];
  const int t = threadIdx.x;
  const int rt = 1023 - t;
  int sum = 0;
  for (int q = 0; q < per; q++) sum += (int)hist[rt * per + q];
  int total;
  int above = block_excl_scan(sum, sh, total);
  const int want = k - ctl->above;
  if (above < want && above + sum >= want) {
    for (int q = per - 1; q >= 0; q--) {
      const int b = rt * per + q;
      const int c = (int)hist[b];
      if (above + c >= want) {
        ctl->thr = ((unsigned)ctl->hi << 16) | (unsigned)b;
        ctl->need = want - above;
        break;
      }
      above += c;
    }
  }
}

__global__ __launch_bounds__(256) void k_fe_ties(const unsigned* __restrict__ key, long long P,
                                                 const FeCtl* __restrict__ ctl, int* __restrict__ tie) {
  const bool all = ctl->all != 0;
  const unsigned thr = ctl->thr;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += (long long)gridDim.x * blockDim.x)
    tie[p] = (!all && key[p] == thr) ? 1 : 0;
}

__device__ __forceinline__ bool fe_kept(unsigned kk, int tie_rank, const FeCtl& c) {
  if (c.all) return kk != 0u;
  return kk > c.thr || (kk == c.thr && tie_rank < c.need);
}

__global__ __launch_bounds__(256) void k_fe_keep(const unsigned* __restrict__ key, const int* __restrict__ tie_rank,
                                                 long long P, const FeCtl* __restrict__ ctl, int* __restrict__ keep) {
  const FeCtl c = *ctl;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += (long long)gridDim.x * blockDim.x)
    keep[p] = fe_kept(key[p], tie_rank[p], c) ? 1 : 0;
}

// The kept pixels' points and labels, at their rank in pixel order.
__global__ __launch_bounds__(256) void k_fe_emit(const float* __restrict__ I, const float* __restrict__ depth,
                                                 const float* __restrict__ rgb, const unsigned* __restrict__ key,
                                                 const int* __restrict__ tie_rank, const int* __restrict__ pos, int W,
                                                 int H, double fx, double fy, double cx, double cy, int k,
                                                 const FeCtl* __restrict__ ctl, float* __restrict__ xyz,
                                                 float* __restrict__ feat) {
  const FeCtl c = *ctl;
  const long long P = (long long)W * H;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += (long long)gridDim.x * blockDim.x) {
    if (!fe_kept(key[p], tie_rank[p], c)) continue;
    const int o = pos[p];
    if (o < 0 || o >= k) continue;  // cannot happen: at most k pixels are kept
    const int v = (int)(p / W), u = (int)(p - (long long)v * W);
    const float d = depth[p];
    const float rx = (float)(((double)u - cx) / fx);
    const float ry = (float)(((double)v - cy) / fy);
    xyz[3 * (size_t)o] = rx * d;
    xyz[3 * (size_t)o + 1] = ry * d;
    xyz[3 * (size_t)o + 2] = d;
    float gu, gv;
    fe_grad(I, W, H, u, v, gu, gv);
    float* f = feat + 5 * (size_t)o;
    f[0] = rgb[3 * p];
    f[1] = rgb[3 * p + 1];
    f[2] = rgb[3 * p + 2];
    f[3] = (float)(0.5 + 0.5 * tanh((double)gu / 0.05));
    f[4] = (float)(0.5 + 0.5 * tanh((double)gv / 0.05));
  }
}

__global__ void k_fe_count(FeCtl* __restrict__ ctl, int k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl->n_out = ctl->all ? ctl->valid : k;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int blocks_for(long long work, int bs, int cap) {
  long long b = (work + bs - 1) / bs;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

// Device memory of the allocation-free evaluation (cvo_eval_static): one
// file-scope array per device, alive until the process ends.  Host code never
// passes the array's name to a kernel (in host code it is a stand-in, not a
// device address); it asks for the device address once per device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch_address(void** ptr) { return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch)); }

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  if (words == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(blocks_for((long long)words, 256, 4096)), dim3(256), 0, s, (unsigned*)p, words);
  return hipGetLastError();
}

hipError_t launch_gather_states(const ReqStatic* reqs, int nreq, ReqState* out, hipStream_t s) {
  if (nreq < 1) return hipSuccess;
  const long long words = (long long)nreq * (long long)(sizeof(ReqState) / 8);
  hipLaunchKernelGGL(k_gather_states, dim3(blocks_for(words, 256, 1024)), dim3(256), 0, s, reqs, nreq, out);
  return hipGetLastError();
}

static void launch_scan(const ScanArgs* args, int nseg, long long maxlen, hipStream_t s) {
  if (maxlen <= kScanTile) {
    hipLaunchKernelGGL(k_scan_single, dim3(1, nseg), dim3(kScanBlock), 0, s, args);
    return;
  }
  const int tiles = (int)((maxlen + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_up, dim3(tiles, nseg), dim3(kScanBlock), 0, s, args);
  hipLaunchKernelGGL(k_scan_mid, dim3(1, nseg), dim3(kScanBlock), 0, s, args);
  hipLaunchKernelGGL(k_scan_down, dim3(tiles, nseg), dim3(kScanBlock), 0, s, args);
}

hipError_t launch_ingest(const IngestArgs& a, hipStream_t s) {
  const int B = 256;
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, a.state, a.T0, a.xi0, a.a2_param);
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(3LL * a.n, B, 1024)), dim3(B), 0, s, a.sx, 3LL * a.n, a.state);
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for((long long)a.fd * a.n, B, 1024)), dim3(B), 0, s, a.sfeat,
                     (long long)a.fd * a.n, a.state);
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(3LL * a.m, B, 1024)), dim3(B), 0, s, a.tx, 3LL * a.m, a.state);
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for((long long)a.fd * a.m, B, 1024)), dim3(B), 0, s, a.tfeat,
                     (long long)a.fd * a.m, a.state);
  hipLaunchKernelGGL(k_bbox_partial, dim3(a.nblk_bbox), dim3(B), 0, s, a.sx, a.n, a.xpart);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kBboxThreads), 0, s, a.xpart, a.nblk_bbox, a.n, a.xbox);
  hipLaunchKernelGGL(k_bbox_partial, dim3(a.nblk_bbox), dim3(B), 0, s, a.tx, a.m, a.zpart);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kBboxThreads), 0, s, a.zpart, a.nblk_bbox, a.m, a.zbox);
  hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(32), 0, s, a.xbox, a.n_stages, a.stage_ell, a.kappa,
                     a.cells_per_reach, a.brute_div, a.kcap, a.grid, a.ncell);
  hipLaunchKernelGGL(k_src_keys, dim3(blocks_for(a.n, B, 1024), a.n_stages), dim3(B), 0, s, a.sx, a.n, a.grid,
                     a.src_keys);
  hipLaunchKernelGGL(k_tgt_keys, dim3(blocks_for(a.m, B, 1024)), dim3(B), 0, s, a.tx, a.m, a.zbox, a.tgt_keys);
  const int nseg = a.n_stages + 1;
  // digits of the largest key range: keys lie below max_kcap
  int bits = 1;
  while (bits < 31 && (1LL << bits) < (long long)a.max_kcap) bits++;
  const int passes = (bits + 7) / 8;
  const int rblocks = (a.max_seg_n + kRadixTile - 1) / kRadixTile;
  for (int p = 0; p < passes; p++) {
    hipLaunchKernelGGL(k_radix_hist, dim3(rblocks, nseg), dim3(kRadixThreads), 0, s, a.segs, p);
    launch_scan(a.sort_scans, nseg, (long long)kRadixBins * rblocks, s);
    hipLaunchKernelGGL(k_radix_scatter, dim3(rblocks, nseg), dim3(kRadixThreads), 0, s, a.segs, p,
                       p == passes - 1 ? 1 : 0);
  }
  hipLaunchKernelGGL(k_radix_start, dim3(blocks_for(a.max_kcap + 1LL, B, 2048), nseg), dim3(B), 0, s, a.segs,
                     passes);
  hipLaunchKernelGGL(k_tgt_records, dim3(blocks_for(a.m, B, 1024)), dim3(B), 0, s, a.tx, a.tfeat, a.m, a.fd, a.zs,
                     a.tgt_perm, a.zrec, a.zorig);
  if (a.precision == 1) {
    hipLaunchKernelGGL(k_src_records<double>, dim3(blocks_for(a.n, B, 1024), a.n_stages), dim3(B), 0, s, a.sx,
                       a.sfeat, a.n, a.fd, a.xs, a.grid, a.src_keys, a.src_perm, (double* const*)a.xrec_dev);
  } else {
    hipLaunchKernelGGL(k_src_records<float>, dim3(blocks_for(a.n, B, 1024), a.n_stages), dim3(B), 0, s, a.sx,
                       a.sfeat, a.n, a.fd, a.xs, a.grid, a.src_keys, a.src_perm, (float* const*)a.xrec_dev);
  }
  // target clusters, one clustering per stage, every stage in each launch
  const int gm = blocks_for(a.m, B, 1024);
  const int S = a.n_stages;
  hipLaunchKernelGGL(k_cl_flags, dim3(gm, S), dim3(B), 0, s, a.zrec, a.zs, a.m, a.zbox, a.kappa, a.stage_ell,
                     a.cl_flag, a.cl_scan);
  launch_scan(a.cl_scan_args, S, a.m, s);
  hipLaunchKernelGGL(k_cl_segfirst, dim3(gm, S), dim3(B), 0, s, a.cl_flag, a.cl_scan, a.m, a.cl_first);
  hipLaunchKernelGGL(k_cl_cflags, dim3(gm, S), dim3(B), 0, s, a.cl_flag, a.cl_scan, a.cl_first, a.m);
  launch_scan(a.cl_scan_args, S, a.m, s);
  hipLaunchKernelGGL(k_cl_table, dim3(gm, S), dim3(B), 0, s, a.cl_flag, a.cl_scan, a.m, a.clus_start, a.state);
  hipLaunchKernelGGL(k_cl_count, dim3(gm, S), dim3(B), 0, s, a.clus_start, a.state, a.m, a.clus_count);
  hipLaunchKernelGGL(k_setup_final, dim3(1), dim3(1), 0, s, a.state, a.xbox, a.zbox, a.a2_param, a.n_stages);
  return hipGetLastError();
}

// Persistent grid of the pair kernel: as many workgroups as are resident at
// once (occupancy of this instance times the compute units), capped by the
// largest item count the launch can have.
static int resident_blocks(const void* kernel, int block_threads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block_threads, 0) != hipSuccess)
    return -1;
  return (per_cu < 1 ? 1 : per_cu) * (cus < 1 ? 1 : cus);
}

template <typename CT, int FD, bool CUT, bool QUART>
static hipError_t launch_pairs3(const ReqStatic* reqs, const int* clus_end, int nreq, int total,
                                const QueueRef& Q, hipStream_t s) {
  static std::atomic<int> resident_cache{0};  // per instance; every device of a process is the same part
  int resident = resident_cache.load(std::memory_order_relaxed);
  if (resident <= 0) {
    resident = resident_blocks((const void*)k_pairs<CT, FD, CUT, QUART>, PairWaves<CT>::value * kWave);
    if (resident <= 0) return hipErrorInvalidValue;
    resident_cache.store(resident, std::memory_order_relaxed);
  }
  const long long most = (long long)Q.cap;
  const int blocks = (int)(most < resident ? most : resident);
  hipLaunchKernelGGL((k_pairs<CT, FD, CUT, QUART>), dim3(blocks), dim3(PairWaves<CT>::value * kWave), 0, s, reqs,
                     clus_end, nreq, Q);
  return hipGetLastError();
}

template <typename CT, int FD>
static hipError_t launch_pairs(bool cut, bool quart, const ReqStatic* reqs, const int* clus_end, int nreq, int total,
                               const QueueRef& Q, hipStream_t s) {
  if (quart)
    return cut ? launch_pairs3<CT, FD, true, true>(reqs, clus_end, nreq, total, Q, s)
               : launch_pairs3<CT, FD, false, true>(reqs, clus_end, nreq, total, Q, s);
  return cut ? launch_pairs3<CT, FD, true, false>(reqs, clus_end, nreq, total, Q, s)
             : launch_pairs3<CT, FD, false, false>(reqs, clus_end, nreq, total, Q, s);
}

template <typename CT>
static hipError_t launch_pairs_fd(int fd, bool cut, bool quart, const ReqStatic* reqs, const int* clus_end, int nreq,
                                  int total, const QueueRef& Q, hipStream_t s) {
  switch (fd) {
    case 1: return launch_pairs<CT, 1>(cut, quart, reqs, clus_end, nreq, total, Q, s);
    case 2: return launch_pairs<CT, 2>(cut, quart, reqs, clus_end, nreq, total, Q, s);
    case 3: return launch_pairs<CT, 3>(cut, quart, reqs, clus_end, nreq, total, Q, s);
    case 4: return launch_pairs<CT, 4>(cut, quart, reqs, clus_end, nreq, total, Q, s);
    case 5: return launch_pairs<CT, 5>(cut, quart, reqs, clus_end, nreq, total, Q, s);
    case 6: return launch_pairs<CT, 6>(cut, quart, reqs, clus_end, nreq, total, Q, s);
    case 7: return launch_pairs<CT, 7>(cut, quart, reqs, clus_end, nreq, total, Q, s);
    default: return launch_pairs<CT, 8>(cut, quart, reqs, clus_end, nreq, total, Q, s);
  }
}

static bool queue_fits(int total_clusters, const QueueRef& Q) {
  return Q.q && Q.items && total_clusters >= 1 && total_clusters < kMaxLaunchClusters &&
         (unsigned long long)total_clusters <= Q.cap;
}

hipError_t launch_prepare(const ReqStatic* reqs, const int* clus_end, int nreq, int total_clusters, const QueueRef& Q,
                          hipStream_t s) {
  if (!queue_fits(total_clusters, Q)) return hipErrorInvalidValue;
  const int blocks = (total_clusters + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(k_prepare, dim3(blocks), dim3(256), 0, s, reqs, clus_end, nreq, total_clusters, Q);
  return hipGetLastError();
}

hipError_t launch_pair_kernel(int precision, int fd, bool cutoff, const ReqStatic* reqs, const int* clus_end, int nreq,
                              int total_clusters, const QueueRef& Q, hipStream_t s) {
  if (fd < 1 || fd > kMaxFeat || !queue_fits(total_clusters, Q)) return hipErrorInvalidValue;
  if (precision == 1) return launch_pairs_fd<double>(fd, cutoff, false, reqs, clus_end, nreq, total_clusters, Q, s);
  return launch_pairs_fd<float>(fd, cutoff, false, reqs, clus_end, nreq, total_clusters, Q, s);
}

hipError_t launch_quartic_pairs(int precision, int fd, bool cutoff, const ReqStatic* reqs, const int* clus_end,
                                int nreq, int total_clusters, const QueueRef& Q, hipStream_t s) {
  if (fd < 1 || fd > kMaxFeat || !queue_fits(total_clusters, Q)) return hipErrorInvalidValue;
  if (precision == 1) return launch_pairs_fd<double>(fd, cutoff, true, reqs, clus_end, nreq, total_clusters, Q, s);
  return launch_pairs_fd<float>(fd, cutoff, true, reqs, clus_end, nreq, total_clusters, Q, s);
}

hipError_t launch_step(const ReqStatic* reqs, const int* clus_end, int nreq, int total_clusters, const QueueRef& Q,
                       hipStream_t s, int phase, bool reset) {
  if (nreq < 1 || !queue_fits(total_clusters, Q)) return hipErrorInvalidValue;
  if (phase != kPhaseFixed && phase != kPhaseGradient && phase != kPhaseQuartic) return hipErrorInvalidValue;
  const int blocks = (total_clusters + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(k_reduce, dim3(blocks), dim3(256), 0, s, reqs, clus_end, nreq, total_clusters, Q,
                     reset ? 1 : 0);
  hipLaunchKernelGGL(k_step, dim3(nreq), dim3(kStepThreads), 0, s, reqs, nreq, phase);
  return hipGetLastError();
}

hipError_t launch_iteration(int precision, int fd, bool cutoff, const ReqStatic* reqs, const int* clus_end, int nreq,
                            int total_clusters, const QueueRef& Q, hipStream_t s) {
  return launch_iteration_rule(kStepFixed, precision, fd, cutoff, reqs, clus_end, nreq, total_clusters, Q, s);
}

hipError_t launch_iteration_rule(int step_rule, int precision, int fd, bool cutoff, const ReqStatic* reqs,
                                 const int* clus_end, int nreq, int total_clusters, const QueueRef& Q, hipStream_t s) {
  hipError_t e = launch_prepare(reqs, clus_end, nreq, total_clusters, Q, s);
  if (e != hipSuccess) return e;
  e = launch_pair_kernel(precision, fd, cutoff, reqs, clus_end, nreq, total_clusters, Q, s);
  if (e != hipSuccess) return e;
  if (step_rule == kStepFixed) return launch_step(reqs, clus_end, nreq, total_clusters, Q, s);
  e = launch_step(reqs, clus_end, nreq, total_clusters, Q, s, kPhaseGradient, false);
  if (e != hipSuccess) return e;
  e = launch_quartic_pairs(precision, fd, cutoff, reqs, clus_end, nreq, total_clusters, Q, s);
  if (e != hipSuccess) return e;
  return launch_step(reqs, clus_end, nreq, total_clusters, Q, s, kPhaseQuartic, true);
}

hipError_t launch_frontend(const FrontendArgs& a, hipStream_t s) {
  const long long P = (long long)a.W * a.H;
  if (a.W < 1 || a.H < 1 || P > (long long)kScanTile * kScanBlock || a.k < 1) return hipErrorInvalidValue;
  const int B = 256;
  const int g = blocks_for(P, B, 2048);
  hipError_t e = launch_zero(a.hist_hi, sizeof(unsigned) * kFeBins, s);
  if (e != hipSuccess) return e;
  e = launch_zero(a.hist_lo, sizeof(unsigned) * kFeBins, s);
  if (e != hipSuccess) return e;
  e = launch_zero(a.ctl, sizeof(FeCtl), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fe_intensity, dim3(g), dim3(B), 0, s, a.rgb, P, a.I, a.ctl);
  hipLaunchKernelGGL(k_fe_score, dim3(g), dim3(B), 0, s, a.I, a.depth, a.W, a.H, a.dmin, a.dmax, a.key, a.hist_hi);
  hipLaunchKernelGGL(k_fe_find, dim3(1), dim3(1024), 0, s, a.hist_hi, a.k, a.ctl);
  hipLaunchKernelGGL(k_fe_hist_lo, dim3(g), dim3(B), 0, s, a.key, P, a.ctl, a.hist_lo);
  hipLaunchKernelGGL(k_fe_find_lo_gate, dim3(1), dim3(1024), 0, s, a.hist_lo, a.k, a.ctl);
  hipLaunchKernelGGL(k_fe_ties, dim3(g), dim3(B), 0, s, a.key, P, a.ctl, a.tie);
  launch_scan(a.scans, 1, P, s);
  hipLaunchKernelGGL(k_fe_keep, dim3(g), dim3(B), 0, s, a.key, a.tie, P, a.ctl, a.pos);
  launch_scan(a.scans + 1, 1, P, s);
  hipLaunchKernelGGL(k_fe_emit, dim3(g), dim3(B), 0, s, a.I, a.depth, a.rgb, a.key, a.tie, a.pos, a.W, a.H, a.fx,
                     a.fy, a.cx, a.cy, a.k, a.ctl, a.xyz, a.feat);
  hipLaunchKernelGGL(k_fe_count, dim3(1), dim3(1), 0, s, a.ctl, a.k);
  return hipGetLastError();
}

}  // namespace cvo
