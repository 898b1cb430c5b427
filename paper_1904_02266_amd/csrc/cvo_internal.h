// Internal structures shared by the HIP kernels and the host driver of the
// continuous-registration library.  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cvo {

constexpr int kMaxStages = 8;
constexpr int kMaxFeat = 8;
constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kWavesPerBlock = 4;   // one work item per wavefront, 256-thread blocks
constexpr int kSlot = 9;            // doubles per partial: W, omega[3], D[3], pairs within, pairs examined
constexpr int kTraceCols = 26;      // F, omega[3], v[3], tau, ell, pairs, T[16] after the step
constexpr int kZBits = 6;           // Morton bits per axis for the target spatial order
constexpr int kZBuckets = 1 << (3 * kZBits);
// Work items: a target cluster's candidate sources are cut into chunks of at
// least chunk_min sources and at most chunks_max chunks (per request, from the
// tuning table or the parameters; these are the defaults and the limits).
constexpr int kChunkMinDefault = 256;  // candidate sources per work item, at least
constexpr int kChunksMaxDefault = 64;  // work items per target cluster, at most
constexpr int kChunkMinLo = 8;
constexpr int kChunksCap = 256;     // the largest chunks_max
constexpr int kItemShift = 8;       // work item = launch-wide cluster index << kItemShift | chunk
static_assert((1 << kItemShift) >= kChunksCap, "chunk index fits the item encoding");
constexpr int kMaxLaunchClusters = 1 << (32 - kItemShift);
constexpr int kPairBlockWaves = 16;  // wavefronts per FP32 pair-kernel workgroup (one workgroup per CU; FP64: 8)
constexpr int kCellCap = 512;       // cell-list entries per cluster; beyond: box enumeration
constexpr int kMaxDim = 2047;       // cells per grid axis (packed coordinates use 11 bits)
constexpr int kStage32 = 128;       // sources staged in LDS per round and wave (FP32 path)
constexpr int kStage64 = 64;        // sources staged in LDS per round and wave (FP64 path)
constexpr int kScanPerThread = 16;  // multi-block scan: elements per thread
constexpr int kScanBlock = 1024;    // multi-block scan: threads per block
constexpr int kScanTile = kScanPerThread * kScanBlock;

enum Mode : int { kModeRegister = 0, kModeEval = 1, kModeEvalTargets = 2, kModeQuartic = 3 };
// Step rules: tau = eta ell^2 / F along the gradient; the maximiser of the
// fourth-order model of G(t) = F(h exp(t d)) (second pair pass) along the
// gradient d = grad F, or along conjugate directions d (Polak-Ribiere with
// restarts, the inner products in the metric a^2, b^2).
enum StepRule : int { kStepFixed = 0, kStepQuartic = 1, kStepConjugate = 2 };
constexpr int kCgRestart = 6;  // conjugate directions restart from the gradient every 6 steps (dim se(3))
// The quartic model is trusted for steps that move a typical target by at
// most this many length-scales.
constexpr double kTrustLengths = 3.0;
// Phases of the step kernel: the whole step (fixed rule); the gradient only
// (first pass of the quartic rule, or of a coefficient evaluation); the
// quartic step from the second pass's sums.
enum StepPhase : int { kPhaseFixed = 0, kPhaseGradient = 1, kPhaseQuartic = 2 };

// Geometry of one source grid (one per length-scale stage), written on the device.
struct GridInfo {
  double ox, oy, oz;  // lower corner of cell (0,0,0)
  double h;           // cell edge (m)
  double sq;          // coordinate scale sqrt(log2(e) / (2 ell^2)): exp2(-|sq d|^2) = exp(-|d|^2/(2 ell^2))
  double ell;
  double reach;       // candidate-cell search radius (m); 0 for brute force
  double rc2s;        // cutoff radius squared in scaled units; +inf for brute force (each pair
                      // type rounds it once: FP64 keeps the cutoff exact to FP64)
  int nx, ny, nz, ncell;
  int cutoff;         // 1: grid culling and per-pair cutoff test
  int pad;
};

// One reachable, non-empty source cell of a target cluster's candidate list.
struct CellEntry {
  int cell;   // cell coordinates packed as cx | cy << 11 | cz << 22
  int first;  // first sorted source of the cell
  int count;  // sources in the cell
  int end;    // inclusive prefix of counts along the list
};

// Per target cluster, rebuilt every iteration by the prepare kernel: the
// frame in which the pair kernel works on the cluster, and its candidates.
// Candidate cell box of a target cluster and its bounding sphere (cells
// lo .. lo + r - 1 per axis; a cell counts only if it is within reach of the
// sphere of centre cc).
struct CandBox {
  int lo0, lo1, lo2, rx, ry, rz, ncand;
  int pad;
  double cc[3];
  double reach2;
};

struct ClusInfo {
  double O[3];        // origin: the centre of the targets' bounding box (m)
  double base[3];     // position of source cell (0,0,0) relative to O, scaled units
  double hs;          // cell edge, scaled units
  double isq;         // 1 / (scale): scaled units -> m
  float blo[3];       // bounding box of the cluster's targets relative to O, scaled units
  float bhi[3];
  const void* xrec;   // source records of the current stage
  int total;          // candidate sources of the cluster
  int ncells;         // list entries (may exceed kCellCap: then overflow)
  int overflow;       // 1: the pair kernel enumerates the candidate box itself
  int nchunks;        // work items of the cluster (1..chunks_max)
  int chunk;          // candidate sources per work item (the last one may hold fewer)
  int s0, cn;         // first sorted target and target count
  int stage;
  CandBox box;        // the candidate box the list was built from (the overflow path enumerates it again)
};

// Work list of one iteration launch: the prepare kernel appends items, each
// persistent workgroup of the pair kernel takes an equal share of the list,
// the step kernel resets the count for the next launch.
struct WorkQueue {
  unsigned int nitems;  // items appended
  unsigned int pad;
};
struct QueueRef {
  WorkQueue* q;
  unsigned int* items;  // [cap]
  unsigned int cap;     // >= sum over the launch's requests of clusters * chunks_max
};

struct ReqState;

// Per-request constants, written by the host before the first launch.
struct ReqStatic {
  ReqState* state;                   // this request's mutable state
  const float* zrec;                 // [m][zs] target xyz (raw FP32) + labels, spatially sorted
  const int* zorig;                  // [m] original index of each sorted target
  const int* clus_start[kMaxStages]; // per stage: [nclus_s] first sorted target of each cluster
  const int* clus_count[kMaxStages]; // per stage: [nclus_s] targets in each cluster (1..64)
  const void* xrec[kMaxStages];      // per stage: [n][xs] scaled cell-local offsets + labels
  const int* cstart[kMaxStages];     // per stage: [ncell+1] first sorted source of each cell
  const GridInfo* grid;              // [n_stages]
  ClusInfo* cinfo;                   // [nclus]
  CellEntry* cells;                  // [nclus][kCellCap]
  int* centry;                       // [nclus][chunks_max] list entry holding each chunk's first candidate
  void* tblk;                        // [nclus][3 + fd][kWave] targets in the cluster frame (scaled, relative
                                     // to O; far away for lanes past the cluster) and labels, pair type
  double* sslots;                    // [nclus][chunks_max][kSlot] work-item partials
  double* csum;                      // [nclus][kSlot] per-cluster sums of the partials
  double* trace;                     // [max_iters][kTraceCols] or null
  double* per_target;                // [m][7] or null (per-target terms, eval-targets mode)
  int m, n, fd, zs, xs, nclus;        // nclus: the largest cluster count over the stages
  int n_stages, max_iters, mode, precision;
  int step_rule;
  int dof_mask;                      // generators the flow moves along: bits 0-2 omega, 3-5 v
  int chunk_min;                     // work items: candidate sources per item at least
  int chunks_max;                    // work items per target cluster at most (<= kChunksCap)
  int stage_len[kMaxStages];         // iterations of stage s at most; last = INT_MAX
  double stage_ell[kMaxStages];
  double s2f;                        // sigma^2 * s_f
  double b2, eta, tol;
  double grad_tol;                   // stop when |(omega, v)| < grad_tol in the last stage (0: off)
  double stage_tol;                  // leave a stage early once |tau d| < stage_tol (0: off)
};

// Per-request mutable state, device-resident for the whole registration.
struct ReqState {
  double T[12];                      // rows 0..2 of the pose acting on target points
  double g[7];                       // F, omega, v at the last evaluated pose
  double xi[6];                      // direction (omega, v) of the second (quartic) pass and of the step
  double gprev[6];                   // the previous iteration's gradient (in the mask), conjugate rule
  double A[5];                       // F and the model coefficients A1..A4 of the last quartic pass
  unsigned long long last_pairs;     // pairs within the cutoff of the last gradient pass
  double a2;                         // rotational metric weight (device-computed default)
  double zrad;                       // root mean square norm of the targets (m)
  double tau;
  unsigned long long pairs_within, pairs_examined;
  int iter, stage, done, status, converged;
  unsigned int reserved;
  int stage_start;                   // iteration at which the current stage began
  int cg_n;                          // conjugate rule: steps since the last restart (0: restart now)
  int cg_stage;                      // conjugate rule: stage of the direction in xi
  int bad_input;                     // set by the finiteness check
  int nclus;                         // target clusters, the largest over the stages (device-computed at ingest)
  int nclus_s[kMaxStages];           // target clusters of each stage
};

// Descriptor of a counting sort over one key segment (one per stage for the
// source grids, one for the target spatial order).
// One segment of the stable key sort (an LSD radix sort over 8-bit digits,
// tiles of kRadixTile elements per block).
constexpr int kRadixBins = 256;
constexpr int kRadixThreads = 256;
constexpr int kRadixRounds = 4;
constexpr int kRadixTile = kRadixThreads * kRadixRounds;
struct SortSeg {
  const int* keys;   // [n]
  const int* nkeys;  // device pointer to K (keys lie in [0, K))
  int* count;        // [Kcap+1] out: start table, count[k] = number of keys below k (k <= K)
  int *key_a, *idx_a, *key_b, *idx_b;  // [n] each: the passes' keys and original indices
  int* hist;         // [kRadixBins][nblocks] digit counts per block, then their exclusive scan
  int* perm;         // [n] stable order: sorted position -> original index
  int* sums;         // scan tile totals of hist
  int n;
  int kcap;
  int nblocks;       // ceil(n / kRadixTile)
};

// Exclusive in-place scan of data[0..len) with len = (lenp ? *lenp : 0) + len0.
struct ScanArgs {
  int* data;
  const int* lenp;
  int len0;
  int* sums;  // [ceil(len / kScanTile)] tile totals
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
  const double* xi0;         // device [6] direction of the quartic pass (kModeQuartic) or null
  const double* stage_ell;   // device [n_stages]
  double *xpart, *zpart, *xbox, *zbox;
  GridInfo* grid;
  int* ncell;
  int* src_keys;             // [n_stages][n]
  int* tgt_keys;             // [m]
  int* src_perm;             // [n_stages][n]
  int* tgt_perm;             // [m]
  SortSeg* segs;             // device [n_stages + 1] (target segment last)
  ScanArgs* sort_scans;      // device [n_stages + 1], over each segment's radix digit counts (hist)
  ScanArgs* cl_scan_args;    // device [n_stages], stage s over cl_scan + s m (m entries)
  int max_seg_n, max_kcap;
  float* zrec;
  int* zorig;
  void* const* xrec_dev;     // device array [n_stages] of record pointers
  // target clustering (one per stage, all stages in each launch): scratch
  // [n_stages][m] each (cl_sums: [n_stages][m/kScanTile + 1]), outputs
  // [n_stages][m]
  int *cl_flag, *cl_scan, *cl_first, *cl_sums;
  int *clus_start, *clus_count;
  ReqState* state;
  int nblk_bbox;
};
hipError_t launch_ingest(const IngestArgs& a, hipStream_t s);

// RGB-D front end: control block of the selection (device) and arguments.
struct FeCtl {
  int valid;       // valid pixels
  int all;         // 1: at most k valid pixels, all kept
  int hi;          // high 16 bits of the k-th largest key
  int above;       // keys above bin hi
  unsigned thr;    // the k-th largest key
  int need;        // pixels with key == thr to keep (the first ones in pixel order)
  int n_out;       // points written
  int bad;         // a colour value is not finite
};
struct FrontendArgs {
  const float *depth, *rgb;  // device [H][W], [H][W][3]
  int W, H, k;
  float dmin, dmax;
  double fx, fy, cx, cy;
  float* I;                  // [P] intensity
  unsigned* key;             // [P]
  unsigned *hist_hi, *hist_lo;  // [65536] each
  int *tie, *pos;            // [P] each (scanned in place)
  ScanArgs* scans;           // device [2]: over tie, over pos
  FeCtl* ctl;
  float *xyz, *feat;         // device outputs [k][3], [k][5]
};
hipError_t launch_frontend(const FrontendArgs& a, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// copies *reqs[k].state to out[k] for k < nreq (one read-back for a batch)
hipError_t launch_gather_states(const ReqStatic* reqs, int nreq, ReqState* out, hipStream_t s);
// The allocation-free evaluation's device array (cvo_eval_static): its size,
// and its device address on the current device.
constexpr size_t kStaticScratchBytes = 64ull << 20;
hipError_t static_scratch_address(void** ptr);
// One gradient-flow iteration (or one evaluation) for a batch of requests that
// share precision, label dimension and cutoff mode.  clus_end[r] is the
// cumulative cluster count of requests 0..r.
// The queue's count must be zero before the first launch on it (the step
// kernel leaves it zero); one queue serves one stream.
hipError_t launch_iteration(int precision, int fd, bool cutoff, const ReqStatic* reqs, const int* clus_end,
                            int nreq, int total_clusters, const QueueRef& Q, hipStream_t s);
// With step_rule == kStepQuartic (all requests of the launch) the iteration
// is prepare, pairs, reduce, gradient, quartic pairs, reduce, quartic step.
hipError_t launch_iteration_rule(int step_rule, int precision, int fd, bool cutoff, const ReqStatic* reqs,
                                 const int* clus_end, int nreq, int total_clusters, const QueueRef& Q, hipStream_t s);
// the kernels of an iteration, separately (for event timing).  reset: the
// reduce kernel clears the work list (the last reduce of an iteration).
hipError_t launch_step(const ReqStatic* reqs, const int* clus_end, int nreq, int total_clusters, const QueueRef& Q,
                       hipStream_t s, int phase = kPhaseFixed, bool reset = true);
hipError_t launch_quartic_pairs(int precision, int fd, bool cutoff, const ReqStatic* reqs, const int* clus_end,
                                int nreq, int total_clusters, const QueueRef& Q, hipStream_t s);
hipError_t launch_prepare(const ReqStatic* reqs, const int* clus_end, int nreq, int total_clusters, const QueueRef& Q,
                          hipStream_t s);
hipError_t launch_pair_kernel(int precision, int fd, bool cutoff, const ReqStatic* reqs, const int* clus_end, int nreq,
                              int total_clusters, const QueueRef& Q, hipStream_t s);

}  // namespace cvo
