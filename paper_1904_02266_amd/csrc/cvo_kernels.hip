// HIP kernels (gfx950) for continuous sensor registration.
//
// Hot path, per gradient-flow iteration (one launch, k_iterate):
//   every wavefront owns one work item = (request, cluster of 64 spatially
//   sorted target points, slice of the candidate source points);
//   z~_j = T z_j in FP64 per lane, cluster bounding box, candidate source
//   cells within the cutoff reach, per-pair FP32 terms
//       d = z~_j - x_i,  r^2,  e = exp(-r^2/(2 l^2)),  c = <l_i, m_j>,
//       W_j += c e,  D_j += c e d
//   with the source point wave-uniform (scalar loads) and the target per lane;
//   compensated (Kahan) FP32 partials per lane, FP64 wave reduction to a
//   fixed slot per work item; the last wavefront of a request to arrive sums
//   its slots in fixed order (FP64), forms F, omega, v (eq. scalar and
//   eq. 3_gradient), and applies the FP64 exponential-map step (eq. step,
//   eq. newstep) to the device-resident pose.
//
// Set-up kernels: bounding boxes and the default a^2 (FP64), source grids per
// length-scale stage (deterministic counting sort by cell), and a Morton
// order of the target points.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "cvo_internal.h"

namespace cvo {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
// inclusive prefix sum over the wave (Hillis-Steele with shuffles)
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int u = __shfl_up(v, o, kWave);
    if (l >= o) v += u;
  }
  return v;
}

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

// out: min xyz, max xyz, mean |p|^2
__global__ void k_bbox_final(const double* __restrict__ part, int nblk, int n, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double r[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
  for (int b = 0; b < nblk; b++) {
    for (int a = 0; a < 3; a++) {
      r[a] = fmin(r[a], part[7 * b + a]);
      r[3 + a] = fmax(r[3 + a], part[7 * b + 3 + a]);
    }
    r[6] += part[7 * b + 6];
  }
  r[6] /= (double)n;
  for (int q = 0; q < 7; q++) out[q] = r[q];
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
    for (int a = 0; a < 3; a++) cells *= floor(ext[a] / h) + 1.0;
    if (cells <= (double)kcap) fits = true;
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
    g.rc2s = (float)(kappa * kappa * LOG2E * 0.5);
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
// 4) deterministic counting sort (blockIdx.y = segment)
//    histogram -> exclusive scan -> scatter with cursors -> rank fix: the final
//    position of point i inside its key is the number of points of the same
//    key with a smaller index, so the order does not depend on atomics.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sort_zero(const SortSeg* __restrict__ segs) {
  const SortSeg S = segs[blockIdx.y];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= S.kcap; k += gridDim.x * blockDim.x) {
    S.count[k] = 0;
    if (k < S.kcap) S.cursor[k] = 0;
  }
}

__global__ __launch_bounds__(256) void k_sort_hist(const SortSeg* __restrict__ segs) {
  const SortSeg S = segs[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < S.n; i += gridDim.x * blockDim.x)
    atomicAdd(&S.count[S.keys[i]], 1);
}

// single workgroup per segment, 1024 threads, over K+1 entries
__global__ __launch_bounds__(1024) void k_sort_scan(const SortSeg* __restrict__ segs) {
  const SortSeg S = segs[blockIdx.y];
  const int K = *S.nkeys;
  const int total = K + 1;
  const int T = blockDim.x;
  const int per = (total + T - 1) / T;
  const int t = threadIdx.x;
  const int b0 = min(t * per, total), b1 = min(b0 + per, total);
  int local = 0;
  for (int k = b0; k < b1; k++) local += (k < K) ? S.count[k] : 0;
  __shared__ int sh[1024];
  sh[t] = local;
  __syncthreads();
  for (int o = 1; o < T; o <<= 1) {
    int v = (t >= o) ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int run = sh[t] - local;  // exclusive
  for (int k = b0; k < b1; k++) {
    const int c = (k < K) ? S.count[k] : 0;
    S.count[k] = run;
    run += c;
  }
}

__global__ __launch_bounds__(256) void k_sort_scatter(const SortSeg* __restrict__ segs) {
  const SortSeg S = segs[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < S.n; i += gridDim.x * blockDim.x) {
    const int k = S.keys[i];
    const int p = S.count[k] + atomicAdd(&S.cursor[k], 1);
    S.tmp[p] = i;
  }
}

__global__ __launch_bounds__(256) void k_sort_rank(const SortSeg* __restrict__ segs) {
  const SortSeg S = segs[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < S.n; i += gridDim.x * blockDim.x) {
    const int k = S.keys[i];
    const int a = S.count[k], b = S.count[k + 1];
    int r = 0;
    for (int q = a; q < b; q++) r += (S.tmp[q] < i) ? 1 : 0;
    S.perm[a + r] = i;
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
// 6) the iteration kernel
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

// All sources of one cell segment [a, b) against the lane's target.
// Returns nothing; counts are kept in scalar registers by the caller.
template <typename CT, int FD, bool CUT>
__device__ __forceinline__ void cell_segment(const CT* __restrict__ xr, int xs, int a, int b, CT zx, CT zy,
                                             CT zz, const CT (&mj)[FD], CT rc2, Acc<CT>& acc,
                                             unsigned long long& within) {
  for (int b0 = a; b0 < b; b0 += kBlock) {
    const int b1 = min(b0 + kBlock, b);
    for (int i = b0; i < b1; i++) {
      const CT* r = xr + (size_t)i * xs;
      const CT dx = zx - r[0];
      const CT dy = zy - r[1];
      const CT dz = zz - r[2];
      const CT r2 = dx * dx + dy * dy + dz * dz;
      bool in = true;
      if (CUT) {
        in = r2 <= rc2;
        const unsigned long long bal = __ballot(in);
        if (bal == 0ull) continue;
        within += (unsigned long long)__popcll(bal);
      }
      const CT e = kexp2(-r2);
      CT c = r[3] * mj[0];
#pragma unroll
      for (int f = 1; f < FD; f++) c += r[3 + f] * mj[f];
      CT w = c * e;
      if (CUT) w = in ? w : (CT)0;
      acc.w += w;
      acc.dx += w * dx;
      acc.dy += w * dy;
      acc.dz += w * dz;
    }
    acc.fold();
  }
}

__device__ __forceinline__ int find_request(const int* __restrict__ item_end, int nreq, int item) {
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (item < item_end[mid]) hi = mid;
    else lo = mid + 1;
  }
  return lo;
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

// The final reduction and step of one request, run by its last-arriving wave.
__device__ void finish_request(const ReqStatic& R, ReqState* __restrict__ S) {
  const int l = lane_id();
  double acc[kSlot];
  for (int q = 0; q < kSlot; q++) acc[q] = 0.0;
  for (int it = l; it < R.n_items; it += kWave) {
    const double* sl = R.slots + (size_t)it * kSlot;
    for (int q = 0; q < kSlot; q++) acc[q] += sl[q];
  }
  for (int q = 0; q < kSlot; q++) acc[q] = wave_sum(acc[q]);
  if (l != 0) return;

  const int stage = S->stage;
  const double ell = R.stage_ell[stage];
  const double il2 = 1.0 / (ell * ell);
  double g[7];
  g[0] = R.s2f * acc[0];
  for (int a = 0; a < 3; a++) {
    g[1 + a] = R.s2f * acc[1 + a] * il2 / S->a2;
    g[4 + a] = R.s2f * acc[4 + a] * il2 / R.b2;
  }
  for (int q = 0; q < 7; q++) S->g[q] = g[q];
  const unsigned long long pairs = (unsigned long long)acc[7];
  S->pairs_within += pairs;
  S->arrive = 0;

  if (R.mode != kModeRegister) {
    S->done = 1;
    return;
  }
  if (!(g[0] > 1e-300)) {
    S->status = -4;  // no pairs in range
    S->done = 1;
    return;
  }
  const double tau = R.eta * ell * ell / g[0];
  S->tau = tau;
  const double w[3] = {-tau * g[1], -tau * g[2], -tau * g[3]};
  const double u[3] = {-tau * g[4], -tau * g[5], -tau * g[6]};
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
    tr[9] = (double)pairs;
    for (int q = 0; q < 12; q++) tr[10 + q] = T[q];
    tr[22] = 0.0;
    tr[23] = 0.0;
    tr[24] = 0.0;
    tr[25] = 1.0;
  }
  double sq = 0.0;
  for (int a = 0; a < 3; a++) sq += w[a] * w[a] + u[a] * u[a];
  const int kn = k + 1;
  S->iter = kn;
  if (stage == R.n_stages - 1 && sqrt(sq) < R.tol) {
    S->converged = 1;
    S->done = 1;
  } else if (kn >= R.max_iters) {
    S->done = 1;
  }
  if (stage < R.n_stages - 1 && kn >= R.stage_end[stage]) S->stage = stage + 1;
}

template <typename CT, int FD, bool CUT>
__global__ __launch_bounds__(256) void k_iterate(const ReqStatic* __restrict__ reqs, const int* __restrict__ item_end,
                                                 int nreq, int total_items) {
  // XCD-aware block order: consecutive logical blocks share an XCD (L2).
  const int nb = gridDim.x;
  const int full = (nb / 8) * 8;
  const int b = blockIdx.x;
  const int lb = (b < full) ? (b % 8) * (full / 8) + b / 8 : b;
  const int item = uniform(lb * kItemsPerBlock + (int)(threadIdx.x >> 6));
  if (item >= total_items) return;
  const int r = uniform(find_request(item_end, nreq, item));
  const ReqStatic& R = reqs[r];
  ReqState* S = R.state;
  if (S->done) return;
  const int local = item - (r > 0 ? item_end[r - 1] : 0);
  const int split = R.split;
  const int clus = local / split;
  const int part = local - clus * split;
  const int l = lane_id();
  const int j = clus * kWave + l;
  const bool valid = j < R.m;

  // target point and labels
  double zt[3] = {0.0, 0.0, 0.0};
  CT mj[FD];
  {
    const double* T = S->T;
    const float* zr = R.zrec + (size_t)(valid ? j : 0) * R.zs;
    const double z0 = zr[0], z1 = zr[1], z2 = zr[2];
#pragma unroll
    for (int f = 0; f < FD; f++) mj[f] = (CT)zr[3 + f];
    for (int a = 0; a < 3; a++) zt[a] = T[4 * a] * z0 + T[4 * a + 1] * z1 + T[4 * a + 2] * z2 + T[4 * a + 3];
  }
  const unsigned long long vmask = __ballot(valid);
  const int nvalid = __popcll(vmask);

  const int stage = S->stage;
  const GridInfo g = R.grid[stage];
  const CT* __restrict__ xr = (const CT*)R.xrec[stage];
  const int* __restrict__ cs = R.cstart[stage];
  const int xs = R.xs;

  // candidate cell box
  int lo[3], hi[3];
  if (g.cutoff) {
    const double o[3] = {g.ox, g.oy, g.oz};
    const int dim[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; a++) {
      const double bmin = wave_min(valid ? zt[a] : INFINITY);
      const double bmax = wave_max(valid ? zt[a] : -INFINITY);
      const double fl = floor((bmin - g.reach - o[a]) / g.h);
      const double fh = floor((bmax + g.reach - o[a]) / g.h);
      // clamp in FP64 before the conversion so that far clusters give empty ranges
      lo[a] = (int)fmin(fmax(fl, 0.0), (double)dim[a]);
      hi[a] = (int)fmax(fmin(fh, (double)(dim[a] - 1)), -1.0);
    }
  } else {
    lo[0] = lo[1] = lo[2] = 0;
    hi[0] = g.nx - 1;
    hi[1] = g.ny - 1;
    hi[2] = g.nz - 1;
  }
  const int rx = uniform(max(hi[0] - lo[0] + 1, 0));
  const int ry = uniform(max(hi[1] - lo[1] + 1, 0));
  const int rz = uniform(max(hi[2] - lo[2] + 1, 0));
  const int ncand = rx * ry * rz;
  const int lo0 = uniform(lo[0]), lo1 = uniform(lo[1]), lo2 = uniform(lo[2]);

  // pass 1: number of candidate sources
  long long total = 0;
  for (int c0 = 0; c0 < ncand; c0 += kWave) {
    const int t = c0 + l;
    int cnt = 0;
    if (t < ncand) {
      const int ix = t % rx, iy = (t / rx) % ry, iz = t / (rx * ry);
      const int key = ((lo2 + iz) * g.ny + (lo1 + iy)) * g.nx + (lo0 + ix);
      cnt = cs[key + 1] - cs[key];
    }
    total += uniform(wave_sum_int(cnt));
  }
  const long long s0 = total * part / split, s1 = total * (part + 1) / split;

  // pass 2: my slice [s0, s1) of the concatenated candidate sources
  Acc<CT> acc;
  acc.init();
  unsigned long long within = 0;
  unsigned long long examined = 0;
  const CT rc2 = (CT)g.rc2s;
  long long base = 0;
  for (int c0 = 0; c0 < ncand && base < s1; c0 += kWave) {
    const int t = c0 + l;
    int key = 0, cnt = 0;
    if (t < ncand) {
      const int ix = t % rx, iy = (t / rx) % ry, iz = t / (rx * ry);
      key = ((lo2 + iz) * g.ny + (lo1 + iy)) * g.nx + (lo0 + ix);
      cnt = cs[key + 1] - cs[key];
    }
    const int incl = wave_incl_scan(cnt);
    const int chunk_total = uniform(__shfl(incl, kWave - 1, kWave));
    // lanes whose cell intersects the slice
    const long long cb = base + incl - cnt, ce = base + incl;
    unsigned long long todo = __ballot(cnt > 0 && ce > s0 && cb < s1);
    while (todo) {
      const int src = __builtin_ctzll(todo);
      todo &= todo - 1ull;
      const int ckey = uniform(__shfl(key, src, kWave));
      const long long cbeg = base + uniform(__shfl(incl - cnt, src, kWave));
      const int ccnt = uniform(__shfl(cnt, src, kWave));
      const int first = uniform(cs[ckey]);
      const long long sb = cbeg > s0 ? cbeg : s0;
      const long long se = (cbeg + ccnt) < s1 ? (cbeg + ccnt) : s1;
      const int a = first + (int)(sb - cbeg);
      const int bnd = first + (int)(se - cbeg);
      const int cx = ckey % g.nx, cy = (ckey / g.nx) % g.ny, cz = ckey / (g.nx * g.ny);
      // lanes past the end of the cloud sit far outside every cell: their
      // pairs fail the cutoff test and their kernel values underflow to 0
      const CT far = (CT)1e30;
      const CT zx = valid ? (CT)((zt[0] - (g.ox + cx * g.h)) * g.sq) : far;
      const CT zy = valid ? (CT)((zt[1] - (g.oy + cy * g.h)) * g.sq) : far;
      const CT zz = valid ? (CT)((zt[2] - (g.oz + cz * g.h)) * g.sq) : far;
      cell_segment<CT, FD, CUT>(xr, xs, a, bnd, zx, zy, zz, mj, rc2, acc, within);
      examined += (unsigned long long)(bnd - a) * (unsigned long long)nvalid;
    }
    base += chunk_total;
  }
  if (!CUT) within = examined;

  double W, Dx, Dy, Dz;
  acc.result(W, Dx, Dy, Dz);
  if (!valid) W = Dx = Dy = Dz = 0.0;
  const double isq = 1.0 / g.sq;
  Dx *= isq;
  Dy *= isq;
  Dz *= isq;
  // omega contribution: sum_i w (x_i x z~_j) = z~_j x D_j with D_j = sum_i w (z~_j - x_i)
  const double ox = zt[1] * Dz - zt[2] * Dy;
  const double oy = zt[2] * Dx - zt[0] * Dz;
  const double oz = zt[0] * Dy - zt[1] * Dx;

  if (R.mode == kModeEvalTargets && R.per_target && valid) {
    const int stg = stage;
    const double ell = R.stage_ell[stg];
    const double il2 = 1.0 / (ell * ell);
    double* o = R.per_target + (size_t)R.zorig[j] * 7;
    o[0] = R.s2f * W;
    o[1] = R.s2f * ox * il2 / S->a2;
    o[2] = R.s2f * oy * il2 / S->a2;
    o[3] = R.s2f * oz * il2 / S->a2;
    o[4] = R.s2f * Dx * il2 / R.b2;
    o[5] = R.s2f * Dy * il2 / R.b2;
    o[6] = R.s2f * Dz * il2 / R.b2;
  }

  const double sW = wave_sum(W), sox = wave_sum(ox), soy = wave_sum(oy), soz = wave_sum(oz);
  const double sDx = wave_sum(Dx), sDy = wave_sum(Dy), sDz = wave_sum(Dz);
  if (l == 0) {
    double* sl = R.slots + (size_t)local * kSlot;
    sl[0] = sW;
    sl[1] = sox;
    sl[2] = soy;
    sl[3] = soz;
    sl[4] = sDx;
    sl[5] = sDy;
    sl[6] = sDz;
    sl[7] = (double)within;
    atomicAdd(&S->pairs_examined, examined);
  }
  __threadfence();
  unsigned int old = 0;
  if (l == 0) old = __hip_atomic_fetch_add(&S->arrive, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
  old = __shfl(old, 0, kWave);
  if (old == (unsigned int)(R.n_items - 1)) {
    __threadfence();
    finish_request(R, S);
  }
}

// ---------------------------------------------------------------------------
// 7) request state set-up
// ---------------------------------------------------------------------------
__global__ void k_init_state(ReqState* __restrict__ S, const double* __restrict__ T0, double a2_param) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int q = 0; q < 12; q++) S->T[q] = T0[q];
  for (int q = 0; q < 7; q++) S->g[q] = 0.0;
  S->a2 = a2_param;
  S->tau = 0.0;
  S->pairs_within = 0ull;
  S->pairs_examined = 0ull;
  S->iter = 0;
  S->stage = 0;
  S->done = 0;
  S->status = 0;
  S->converged = 0;
  S->arrive = 0u;
  S->bad_input = 0;
  S->pad = 0;
}

__global__ __launch_bounds__(256) void k_check_finite(const float* __restrict__ p, long long count,
                                                      ReqState* __restrict__ S) {
  bool bad = false;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    bad |= !isfinite(p[i]);
  if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(&S->bad_input, 1);
}

__global__ void k_setup_final(ReqState* __restrict__ S, const double* __restrict__ xbox, double a2_param) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (!(a2_param > 0.0)) S->a2 = xbox[6];
  if (S->bad_input || !(S->a2 > 0.0) || !isfinite(S->a2)) {
    S->status = -1;  // invalid input
    S->done = 1;
  }
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

hipError_t launch_ingest(const IngestArgs& a, hipStream_t s) {
  const int B = 256;
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, a.state, a.T0, a.a2_param);
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(3LL * a.n, B, 1024)), dim3(B), 0, s, a.sx, 3LL * a.n, a.state);
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for((long long)a.fd * a.n, B, 1024)), dim3(B), 0, s, a.sfeat,
                     (long long)a.fd * a.n, a.state);
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for(3LL * a.m, B, 1024)), dim3(B), 0, s, a.tx, 3LL * a.m, a.state);
  hipLaunchKernelGGL(k_check_finite, dim3(blocks_for((long long)a.fd * a.m, B, 1024)), dim3(B), 0, s, a.tfeat,
                     (long long)a.fd * a.m, a.state);
  hipLaunchKernelGGL(k_bbox_partial, dim3(a.nblk_bbox), dim3(B), 0, s, a.sx, a.n, a.xpart);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(1), 0, s, a.xpart, a.nblk_bbox, a.n, a.xbox);
  hipLaunchKernelGGL(k_bbox_partial, dim3(a.nblk_bbox), dim3(B), 0, s, a.tx, a.m, a.zpart);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(1), 0, s, a.zpart, a.nblk_bbox, a.m, a.zbox);
  hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(32), 0, s, a.xbox, a.n_stages, a.stage_ell, a.kappa,
                     a.cells_per_reach, a.brute_div, a.kcap, a.grid, a.ncell);
  hipLaunchKernelGGL(k_src_keys, dim3(blocks_for(a.n, B, 1024), a.n_stages), dim3(B), 0, s, a.sx, a.n, a.grid,
                     a.src_keys);
  hipLaunchKernelGGL(k_tgt_keys, dim3(blocks_for(a.m, B, 1024)), dim3(B), 0, s, a.tx, a.m, a.zbox, a.tgt_keys);
  const int nseg = a.n_stages + 1;
  hipLaunchKernelGGL(k_sort_zero, dim3(blocks_for(a.max_kcap + 1LL, B, 2048), nseg), dim3(B), 0, s, a.segs);
  hipLaunchKernelGGL(k_sort_hist, dim3(blocks_for(a.max_seg_n, B, 1024), nseg), dim3(B), 0, s, a.segs);
  hipLaunchKernelGGL(k_sort_scan, dim3(1, nseg), dim3(1024), 0, s, a.segs);
  hipLaunchKernelGGL(k_sort_scatter, dim3(blocks_for(a.max_seg_n, B, 1024), nseg), dim3(B), 0, s, a.segs);
  hipLaunchKernelGGL(k_sort_rank, dim3(blocks_for(a.max_seg_n, B, 1024), nseg), dim3(B), 0, s, a.segs);
  hipLaunchKernelGGL(k_tgt_records, dim3(blocks_for(a.m, B, 1024)), dim3(B), 0, s, a.tx, a.tfeat, a.m, a.fd, a.zs,
                     a.tgt_perm, a.zrec, a.zorig);
  if (a.precision == 1) {
    hipLaunchKernelGGL(k_src_records<double>, dim3(blocks_for(a.n, B, 1024), a.n_stages), dim3(B), 0, s, a.sx,
                       a.sfeat, a.n, a.fd, a.xs, a.grid, a.src_keys, a.src_perm, (double* const*)a.xrec_dev);
  } else {
    hipLaunchKernelGGL(k_src_records<float>, dim3(blocks_for(a.n, B, 1024), a.n_stages), dim3(B), 0, s, a.sx,
                       a.sfeat, a.n, a.fd, a.xs, a.grid, a.src_keys, a.src_perm, (float* const*)a.xrec_dev);
  }
  hipLaunchKernelGGL(k_setup_final, dim3(1), dim3(1), 0, s, a.state, a.xbox, a.a2_param);
  return hipGetLastError();
}

template <typename CT, int FD>
static void launch_it(bool cut, int blocks, const ReqStatic* reqs, const int* item_end, int nreq, int total,
                      hipStream_t s) {
  if (cut)
    hipLaunchKernelGGL((k_iterate<CT, FD, true>), dim3(blocks), dim3(256), 0, s, reqs, item_end, nreq, total);
  else
    hipLaunchKernelGGL((k_iterate<CT, FD, false>), dim3(blocks), dim3(256), 0, s, reqs, item_end, nreq, total);
}

template <typename CT>
static void launch_fd(int fd, bool cut, int blocks, const ReqStatic* reqs, const int* item_end, int nreq,
                      int total, hipStream_t s) {
  switch (fd) {
    case 1: launch_it<CT, 1>(cut, blocks, reqs, item_end, nreq, total, s); break;
    case 2: launch_it<CT, 2>(cut, blocks, reqs, item_end, nreq, total, s); break;
    case 3: launch_it<CT, 3>(cut, blocks, reqs, item_end, nreq, total, s); break;
    case 4: launch_it<CT, 4>(cut, blocks, reqs, item_end, nreq, total, s); break;
    case 5: launch_it<CT, 5>(cut, blocks, reqs, item_end, nreq, total, s); break;
    case 6: launch_it<CT, 6>(cut, blocks, reqs, item_end, nreq, total, s); break;
    case 7: launch_it<CT, 7>(cut, blocks, reqs, item_end, nreq, total, s); break;
    default: launch_it<CT, 8>(cut, blocks, reqs, item_end, nreq, total, s); break;
  }
}

hipError_t launch_iterate(int precision, int fd, bool cutoff, int blocks, const ReqStatic* reqs,
                          const int* item_end, int nreq, int total_items, hipStream_t s) {
  if (fd < 1 || fd > kMaxFeat || blocks < 1) return hipErrorInvalidValue;
  if (precision == 1)
    launch_fd<double>(fd, cutoff, blocks, reqs, item_end, nreq, total_items, s);
  else
    launch_fd<float>(fd, cutoff, blocks, reqs, item_end, nreq, total_items, s);
  return hipGetLastError();
}

}  // namespace cvo
