// Internal structures shared by the HIP kernels and the host driver of the
// continuous-registration library.  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cvo {

constexpr int kMaxStages = 8;
constexpr int kMaxFeat = 8;
constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kItemsPerBlock = 4;   // one work item per wavefront, 256-thread blocks
constexpr int kSlot = 8;            // doubles per work-item partial: W, omega[3], D[3], pairs
constexpr int kTraceCols = 26;      // F, omega[3], v[3], tau, ell, pairs, T[16] after the step
constexpr int kZBits = 6;           // Morton bits per axis for the target spatial order
constexpr int kZBuckets = 1 << (3 * kZBits);

enum Mode : int { kModeRegister = 0, kModeEval = 1, kModeEvalTargets = 2 };

// Geometry of one source grid (one per length-scale stage), written on the device.
struct GridInfo {
  double ox, oy, oz;  // lower corner of cell (0,0,0)
  double h;           // cell edge (m)
  double sq;          // coordinate scale sqrt(log2(e) / (2 ell^2)): exp2(-|sq d|^2) = exp(-|d|^2/(2 ell^2))
  double ell;
  double reach;       // candidate-cell search radius (m); 0 for brute force
  float rc2s;         // cutoff radius squared in scaled units; +inf for brute force
  int nx, ny, nz, ncell;
  int cutoff;         // 1: grid culling and per-pair cutoff test
  int pad;
};

struct ReqState;

// Per-request constants, written by the host before the first launch.
struct ReqStatic {
  ReqState* state;                   // this request's mutable state
  const float* zrec;                 // [m][zs] target xyz (raw FP32) + labels, spatially sorted
  const int* zorig;                  // [m] original index of each sorted target
  const void* xrec[kMaxStages];      // per stage: [n][xs] scaled cell-local offsets + labels
  const int* cstart[kMaxStages];     // per stage: [ncell+1] first sorted source of each cell
  const GridInfo* grid;              // [n_stages]
  double* slots;                     // [n_items][kSlot]
  double* trace;                     // [max_iters][kTraceCols] or null
  double* per_target;                // [m][7] or null (per-target terms, eval-targets mode)
  int m, n, fd, zs, xs;
  int nclus, split, n_items;         // work items = nclus * split
  int n_stages, max_iters, mode, precision;
  int stage_end[kMaxStages];         // iteration index where stage s ends; last = INT_MAX
  double stage_ell[kMaxStages];
  double s2f;                        // sigma^2 * s_f
  double b2, eta, tol;
};

// Per-request mutable state, device-resident for the whole registration.
struct ReqState {
  double T[12];                      // rows 0..2 of the pose acting on target points
  double g[7];                       // F, omega, v at the last evaluated pose
  double a2;                         // rotational metric weight (device-computed default)
  double tau;
  unsigned long long pairs_within, pairs_examined;
  int iter, stage, done, status, converged;
  unsigned int arrive;               // arrivals of work items in the current launch
  int bad_input;                     // set by the finiteness check
  int pad;
};

// Descriptor of a counting sort over one key segment (one per stage for the
// source grids, one for the target spatial order).
struct SortSeg {
  const int* keys;   // [n]
  const int* nkeys;  // device pointer to K (keys lie in [0, K))
  int* count;        // [Kcap+1] histogram, then exclusive scan (start table)
  int* cursor;       // [Kcap] scatter cursors
  int* tmp;          // [n] scatter output (arbitrary order within a key)
  int* perm;         // [n] stable order: sorted position -> original index
  int n;
  int kcap;
};

// ---------------------------------------------------------------------------
// launchers (defined next to the kernels)
// ---------------------------------------------------------------------------
struct IngestArgs {
  const float *sx, *sfeat, *tx, *tfeat;
  int n, m, fd, zs, xs, n_stages, precision;
  double kappa;
  int cells_per_reach, brute_div, kcap;
  double a2_param;
  const double* T0;          // device [16]
  const double* stage_ell;   // device [n_stages]
  double *xpart, *zpart, *xbox, *zbox;
  GridInfo* grid;
  int* ncell;
  int* src_keys;             // [n_stages][n]
  int* tgt_keys;             // [m]
  int* src_perm;             // [n_stages][n]
  int* tgt_perm;             // [m]
  SortSeg* segs;             // device [n_stages + 1] (target segment last)
  int max_seg_n, max_kcap;
  float* zrec;
  int* zorig;
  void* const* xrec_dev;     // device array [n_stages] of record pointers
  ReqState* state;
  int nblk_bbox;
};
hipError_t launch_ingest(const IngestArgs& a, hipStream_t s);
hipError_t launch_iterate(int precision, int fd, bool cutoff, int blocks, const ReqStatic* reqs,
                          const int* item_end, int nreq, int total_items, hipStream_t s);

}  // namespace cvo
