/*
 * FP64 CPU oracle for continuous sensor registration (Ghaffari et al.,
 * "Continuous Direct Sparse Visual Odometry from RGB-D Images").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow definition that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the library never does.
 * It shares no code, header or constant with the GPU path.
 *
 * Everything is FP64.  Point coordinates and labels arrive as FP32 and are
 * promoted exactly.  Every pair (i, j) is enumerated (brute force); with a
 * cutoff kappa > 0 a pair contributes only if |x_i - z~_j|^2 <= (kappa*ell)^2.
 * For large clouds cvo_oracle_eval_grid enumerates the same cutoff pairs
 * through a uniform source grid (the oracle's own, pinned against the brute
 * force: identical pair set, sums equal to rounding).
 *
 * Notation (paper, Sections III-IV and VI):
 *   X = {x_i}, labels l_i;  Z = {z_j}, labels m_j.
 *   h = (R_h, t_h) in SE(3) is the paper's pose; the paper evaluates the
 *   objective at z~_j = h^-1 z_j = R_h^T z_j - R_h^T t_h (gradient at h).
 *   The library's pose T acts on target points, so T = h^-1.
 *   c_ij = s_f <l_i, m_j>           (label inner product, Sec. VII-B remark)
 *   k_ij = sigma^2 exp(-|x_i - z~_j|^2 / (2 ell^2))   (Sec. IV kernel)
 *   F    = sum_ij c_ij k_ij         (eq. scalar, Problem 1)
 *   omega = 1/(a^2 ell^2) sum_ij c_ij k_ij (x_i x z~_j)      (eq. 3_gradient)
 *   v     = 1/(b^2 ell^2) sum_ij c_ij k_ij (z~_j - x_i)      (eq. 3_gradient,
 *           sign as obtained by differentiating the kernel; the printed
 *           x_i - z~_j has the opposite sign, see the reading list)
 *   step:  h <- h exp(t (omega^, v)), i.e. R <- R dR, t <- R dT + t
 *          (eq. newstep), dR, dT from the closed-form SE(3) exponential
 *          (eq. step), with the step length either t = eta ell^2 / F (project
 *          rule) or the maximiser of the fourth-order Taylor model of
 *          G(t) = F(h exp(t xi)) (Sec. VI-B, eq. fourth; see the quartic
 *          section below for the coefficients used).
 *
 * parity pins: see the oracle tests (finite differences along the six
 * generators, rigid-motion invariance, zero gradient at identical clouds,
 * two-point closed forms, matrix-exponential library routine, recovery).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOOVERLAP (-4)


static void pose_to_inverse_action(const double h[16], double Rt[9], double tt[3]) {
    /* h = [R t; 0 1]; h^-1 z = R^T z - R^T t */
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) Rt[3 * r + c] = h[4 * c + r];
    for (int r = 0; r < 3; r++) {
        double s = 0.0;
        for (int c = 0; c < 3; c++) s += Rt[3 * r + c] * h[4 * c + 3];
        tt[r] = -s;
    }
}

/* Source grid of the enumeration mode (see cvo_oracle_eval_grid): uniform
 * cubic cells of edge h over the source bounding box; the sources of cell k
 * are idx[start[k] .. start[k+1]), in increasing source index. */
typedef struct {
    double o[3], h;
    int dim[3];
    int* start;
    int* idx;
} sgrid_t;

typedef struct {
    int n, m, fd;
    const float *x, *lx, *z, *lz;
    double sigma, sf, ell, kappa, a2, b2;
    double Rt[9], tt[3]; /* z~ = Rt z + tt  (Rt = R_h^T, tt = -R_h^T t_h) */
    int j0, j1;
    const sgrid_t* grid; /* NULL: every source is a candidate of every target */
    /* per-target outputs (optional) */
    const int *sel;
    double *per_target; /* [nsel][7] */
    /* results */
    double sum[7], abs_sum[7];
    long long within, examined;
} job_t;

/* One pair (i, j): adds its terms to s7 and |terms| to a7 if it is inside the
 * cutoff; returns 1 then, 0 otherwise. */
static int pair_terms(const job_t* J, int i, int j, const double zt[3], double s7[7], double a7[7]) {
    const double inv2l2 = 1.0 / (2.0 * J->ell * J->ell);
    const double rc2 = (J->kappa > 0.0) ? (J->kappa * J->ell) * (J->kappa * J->ell) : INFINITY;
    const double s2 = J->sigma * J->sigma;
    const double cw = 1.0 / (J->a2 * J->ell * J->ell);
    const double cv = 1.0 / (J->b2 * J->ell * J->ell);
    const double x0 = J->x[3 * i], x1 = J->x[3 * i + 1], x2 = J->x[3 * i + 2];
    const double d0 = zt[0] - x0, d1 = zt[1] - x1, d2 = zt[2] - x2;
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (!(r2 <= rc2)) return 0;
    double lm = 0.0;
    for (int f = 0; f < J->fd; f++) lm += (double)J->lx[J->fd * i + f] * (double)J->lz[J->fd * j + f];
    const double cij = J->sf * lm;
    const double kij = s2 * exp(-r2 * inv2l2);
    const double w = cij * kij;
    /* x_i cross z~_j */
    const double c0 = x1 * zt[2] - x2 * zt[1];
    const double c1 = x2 * zt[0] - x0 * zt[2];
    const double c2 = x0 * zt[1] - x1 * zt[0];
    const double t[7] = {w, cw * w * c0, cw * w * c1, cw * w * c2, cv * w * d0, cv * w * d1, cv * w * d2};
    for (int q = 0; q < 7; q++) { s7[q] += t[q]; a7[q] += fabs(t[q]); }
    return 1;
}

/* cell coordinate of u along one axis, or a value outside [0, dim) */
static long grid_coord(const sgrid_t* G, int a, double u) {
    const double c = floor((u - G->o[a]) / G->h);
    if (!(c > -2.0)) return -2;
    if (!(c < (double)G->dim[a] + 1.0)) return (long)G->dim[a] + 1;
    return (long)c;
}

/* Terms of the double sum for one target point j, over all sources i (or,
 * with a grid, over the sources of the 27 cells around z~_j: every source
 * within the cutoff lies there, see cvo_oracle_eval_grid).  *examined counts
 * the candidates tested. */
static void target_terms(const job_t* J, int j, double s7[7], double a7[7], long long* within,
                         long long* examined) {
    const double zx = J->z[3 * j], zy = J->z[3 * j + 1], zz = J->z[3 * j + 2];
    double zt[3];
    for (int r = 0; r < 3; r++)
        zt[r] = J->Rt[3 * r] * zx + J->Rt[3 * r + 1] * zy + J->Rt[3 * r + 2] * zz + J->tt[r];
    for (int q = 0; q < 7; q++) { s7[q] = 0.0; a7[q] = 0.0; }
    long long cnt = 0, ex = 0;
    const sgrid_t* G = J->grid;
    if (!G) {
        for (int i = 0; i < J->n; i++) cnt += pair_terms(J, i, j, zt, s7, a7);
        ex = J->n;
    } else {
        long lo[3], hi[3];
        for (int a = 0; a < 3; a++) {
            const long c = grid_coord(G, a, zt[a]);
            lo[a] = c - 1 < 0 ? 0 : c - 1;
            hi[a] = c + 1 > G->dim[a] - 1 ? G->dim[a] - 1 : c + 1;
        }
        for (long cz = lo[2]; cz <= hi[2]; cz++)
            for (long cy = lo[1]; cy <= hi[1]; cy++)
                for (long cx = lo[0]; cx <= hi[0]; cx++) {
                    const long k = (cz * G->dim[1] + cy) * G->dim[0] + cx;
                    for (int p = G->start[k]; p < G->start[k + 1]; p++) {
                        cnt += pair_terms(J, G->idx[p], j, zt, s7, a7);
                        ex++;
                    }
                }
    }
    *within = cnt;
    *examined = ex;
}

static void* run_job(void* arg) {
    job_t* J = (job_t*)arg;
    for (int q = 0; q < 7; q++) { J->sum[q] = 0.0; J->abs_sum[q] = 0.0; }
    J->within = 0; J->examined = 0;
    for (int jj = J->j0; jj < J->j1; jj++) {
        const int j = J->sel ? J->sel[jj] : jj;
        double s7[7], a7[7];
        long long w, ex;
        target_terms(J, j, s7, a7, &w, &ex);
        for (int q = 0; q < 7; q++) { J->sum[q] += s7[q]; J->abs_sum[q] += a7[q]; }
        J->within += w;
        J->examined += ex;
        if (J->per_target)
            for (int q = 0; q < 7; q++) J->per_target[7 * jj + q] = s7[q];
    }
    return NULL;
}

static int check_cloud(int n, int fd, const float* x, const float* l) {
    if (n <= 0 || fd < 1 || fd > 8 || !x || !l) return 0;
    for (long k = 0; k < 3L * n; k++) if (!isfinite(x[k])) return 0;
    for (long k = 0; k < (long)fd * n; k++) if (!isfinite(l[k])) return 0;
    return 1;
}

/* Mean squared norm of the source points (the default a^2), FP64. */
double cvo_oracle_mean_sqnorm(int n, const float* x) {
    double s = 0.0;
    for (int i = 0; i < n; i++) {
        const double a = x[3 * i], b = x[3 * i + 1], c = x[3 * i + 2];
        s += a * a + b * b + c * c;
    }
    return s / (double)n;
}

/*
 * Objective and gradient at the paper's pose h (row-major 4x4).
 *   out[7]    = F, omega[3], v[3]
 *   absout[7] = the same sums with every term replaced by its absolute value
 *   counts[2] = pairs inside the cutoff, pairs examined
 * If sel != NULL only targets sel[0..nsel) are summed and per_target[nsel][7]
 * (optional) receives each target's own terms.  nthreads >= 1 splits the
 * targets into contiguous blocks whose partials are added in block order.
 */
/*
 * Grid enumeration of the same cutoff sum.  Cells are cubes of edge
 * e >= kappa ell (1 + 1e-7) over the sources' bounding box, cell coordinate
 * floor((x_a - o_a) / e) per axis.  A pair within the cutoff has
 * |x_a - z~_a| <= kappa ell < e on every axis, so the two cell coordinates
 * differ by at most one (with at most 2^20 cells per axis the rounding of the
 * divisions stays below 1e-9, far inside the 1e-7 margin): the 27 cells
 * around z~_j hold every source the brute-force enumeration would accept,
 * and each candidate meets the same per-pair test.  The edge grows when the
 * table would exceed 2^26 cells or 2^20 per axis.  Returns 0 on success
 * (free with free_grid).
 */
static int build_grid(int n, const float* x, double edge, sgrid_t* G) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) {
            lo[a] = fmin(lo[a], (double)x[3 * i + a]);
            hi[a] = fmax(hi[a], (double)x[3 * i + a]);
        }
    for (;;) {
        double cells = 1.0, most = 0.0;
        for (int a = 0; a < 3; a++) {
            const double d = floor((hi[a] - lo[a]) / edge) + 1.0;
            cells *= d;
            most = fmax(most, d);
        }
        if (cells <= 67108864.0 && most <= 1048576.0) break;
        edge *= 1.5;
    }
    G->h = edge;
    long ncell = 1;
    for (int a = 0; a < 3; a++) {
        G->o[a] = lo[a];
        G->dim[a] = (int)floor((hi[a] - lo[a]) / edge) + 1;
        ncell *= G->dim[a];
    }
    G->start = (int*)calloc((size_t)ncell + 1, sizeof(int));
    G->idx = (int*)malloc((size_t)n * sizeof(int));
    long* key = (long*)malloc((size_t)n * sizeof(long));
    int* cur = (int*)malloc((size_t)ncell * sizeof(int));
    if (!G->start || !G->idx || !key || !cur) {
        free(G->start); free(G->idx); free(key); free(cur);
        return -1;
    }
    for (int i = 0; i < n; i++) {
        long c[3];
        for (int a = 0; a < 3; a++) {
            c[a] = grid_coord(G, a, (double)x[3 * i + a]);
            if (c[a] < 0) c[a] = 0;
            if (c[a] > G->dim[a] - 1) c[a] = G->dim[a] - 1;
        }
        key[i] = (c[2] * G->dim[1] + c[1]) * G->dim[0] + c[0];
        G->start[key[i] + 1]++;
    }
    for (long k = 0; k < ncell; k++) G->start[k + 1] += G->start[k];
    for (long k = 0; k < ncell; k++) cur[k] = G->start[k];
    for (int i = 0; i < n; i++) G->idx[cur[key[i]]++] = i;
    free(key);
    free(cur);
    return 0;
}

static void free_grid(sgrid_t* G) {
    free(G->start);
    free(G->idx);
}

static int eval_h_impl(int n, const float* x, const float* lx, int m, const float* z, const float* lz,
                       int fd, double sigma, double feat_scale, double ell, double kappa, double a2,
                       double b2, const double h[16], int nsel, const int* sel, int nthreads,
                       double out[7], double absout[7], long long counts[2], double* per_target,
                       int use_grid) {
    if (!check_cloud(n, fd, x, lx) || !check_cloud(m, fd, z, lz)) return OR_EINVAL;
    if (!(ell > 0.0) || !(a2 > 0.0) || !(b2 > 0.0) || kappa < 0.0) return OR_EINVAL;
    if (use_grid && !(kappa > 0.0)) return OR_EINVAL;
    sgrid_t grid;
    if (use_grid && build_grid(n, x, kappa * ell * (1.0 + 1e-7), &grid) != 0) return OR_EINVAL;
    const int nt_total = sel ? nsel : m;
    if (sel)
        for (int k = 0; k < nsel; k++) if (sel[k] < 0 || sel[k] >= m) return OR_EINVAL;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > nt_total) nthreads = nt_total > 0 ? nt_total : 1;
    job_t* jobs = (job_t*)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs); free(th);
        if (use_grid) free_grid(&grid);
        return OR_EINVAL;
    }
    for (int k = 0; k < nthreads; k++) {
        job_t* J = &jobs[k];
        J->grid = use_grid ? &grid : NULL;
        J->n = n; J->m = m; J->fd = fd; J->x = x; J->lx = lx; J->z = z; J->lz = lz;
        J->sigma = sigma; J->sf = feat_scale; J->ell = ell; J->kappa = kappa; J->a2 = a2; J->b2 = b2;
        pose_to_inverse_action(h, J->Rt, J->tt);
        J->j0 = (int)((long long)nt_total * k / nthreads);
        J->j1 = (int)((long long)nt_total * (k + 1) / nthreads);
        J->sel = sel; J->per_target = per_target;
    }
    for (int k = 1; k < nthreads; k++) pthread_create(&th[k], NULL, run_job, &jobs[k]);
    run_job(&jobs[0]);
    for (int k = 1; k < nthreads; k++) pthread_join(th[k], NULL);
    for (int q = 0; q < 7; q++) { out[q] = 0.0; absout[q] = 0.0; }
    counts[0] = counts[1] = 0;
    for (int k = 0; k < nthreads; k++) {
        for (int q = 0; q < 7; q++) { out[q] += jobs[k].sum[q]; absout[q] += jobs[k].abs_sum[q]; }
        counts[0] += jobs[k].within; counts[1] += jobs[k].examined;
    }
    free(jobs); free(th);
    if (use_grid) free_grid(&grid);
    return OR_OK;
}

int cvo_oracle_eval_h(int n, const float* x, const float* lx, int m, const float* z, const float* lz,
                      int fd, double sigma, double feat_scale, double ell, double kappa, double a2,
                      double b2, const double h[16], int nsel, const int* sel, int nthreads,
                      double out[7], double absout[7], long long counts[2], double* per_target) {
    return eval_h_impl(n, x, lx, m, z, lz, fd, sigma, feat_scale, ell, kappa, a2, b2, h, nsel, sel, nthreads,
                       out, absout, counts, per_target, 0);
}

/* Closed-form SE(3) exponential (eq. step) of the twist t*(w^, u), t = 1:
 *   dR = I + (sin th/th) w^ + ((1-cos th)/th^2) w^2
 *   dT = [I + ((1-cos th)/th^2) w^ + ((th - sin th)/th^3) w^2] u,  th = |w|.
 * (1 - cos th) is evaluated as 2 sin^2(th/2), the same quantity without the
 * cancellation of 1 - cos th near 0 (which would leave an absolute error of
 * about eps*|u|/th in dT).  For th < 1e-3 the three coefficients use their
 * Taylor series through th^6 (truncation below 1e-29). */
void cvo_oracle_expmap(const double w[3], const double u[3], double dR[9], double dT[3]) {
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = sqrt(th2);
    double A, B, C;
    if (th < 1e-3) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0 - th2 * th2 * th2 / 5040.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0 - th2 * th2 * th2 / 40320.0;
        C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0 - th2 * th2 * th2 / 362880.0;
    } else {
        const double sh = sin(0.5 * th);
        A = sin(th) / th;
        B = 2.0 * sh * sh / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    const double W[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    double W2[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += W[3 * r + k] * W[3 * k + c];
            W2[3 * r + c] = s;
        }
    double V[9];
    for (int k = 0; k < 9; k++) {
        const double I = (k % 4 == 0) ? 1.0 : 0.0;
        dR[k] = I + A * W[k] + B * W2[k];
        V[k] = I + B * W[k] + C * W2[k];
    }
    for (int r = 0; r < 3; r++) dT[r] = V[3 * r] * u[0] + V[3 * r + 1] * u[1] + V[3 * r + 2] * u[2];
}

/* h <- h exp(t xi): R <- R dR, t_h <- R dT + t_h (eq. newstep). */
static void newstep(double h[16], const double w[3], const double u[3], double t) {
    double tw[3] = {t * w[0], t * w[1], t * w[2]}, tu[3] = {t * u[0], t * u[1], t * u[2]};
    double dR[9], dT[3];
    cvo_oracle_expmap(tw, tu, dR, dT);
    double R[9], tr[3];
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) R[3 * r + c] = h[4 * r + c];
        tr[r] = h[4 * r + 3];
    }
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += R[3 * r + k] * dR[3 * k + c];
            h[4 * r + c] = s;
        }
        h[4 * r + 3] = R[3 * r] * dT[0] + R[3 * r + 1] * dT[1] + R[3 * r + 2] * dT[2] + tr[r];
    }
    h[12] = h[13] = h[14] = 0.0;
    h[15] = 1.0;
}

static void rigid_inverse(const double A[16], double B[16]) {
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) B[4 * r + c] = A[4 * c + r];
        B[4 * r + 3] = -(A[r] * A[3] + A[4 + r] * A[7] + A[8 + r] * A[11]);
    }
    B[12] = B[13] = B[14] = 0.0;
    B[15] = 1.0;
}

/* Same objective, evaluated at the library's convention T = h^-1. */
int cvo_oracle_eval(int n, const float* x, const float* lx, int m, const float* z, const float* lz,
                    int fd, double sigma, double feat_scale, double ell, double kappa, double a2,
                    double b2, const double T[16], int nsel, const int* sel, int nthreads,
                    double out[7], double absout[7], long long counts[2], double* per_target) {
    double h[16];
    rigid_inverse(T, h);
    return cvo_oracle_eval_h(n, x, lx, m, z, lz, fd, sigma, feat_scale, ell, kappa, a2, b2, h, nsel,
                             sel, nthreads, out, absout, counts, per_target);
}

/* The cutoff sum of cvo_oracle_eval (kappa > 0 required) with the candidates
 * of each target taken from a uniform source grid (build_grid) instead of all
 * sources: the same pair set and the same per-pair arithmetic; only the order
 * of the sources inside a target's sum differs.  counts[1] is the number of
 * candidates tested. */
int cvo_oracle_eval_grid(int n, const float* x, const float* lx, int m, const float* z, const float* lz,
                         int fd, double sigma, double feat_scale, double ell, double kappa, double a2,
                         double b2, const double T[16], int nsel, const int* sel, int nthreads,
                         double out[7], double absout[7], long long counts[2], double* per_target) {
    double h[16];
    rigid_inverse(T, h);
    return eval_h_impl(n, x, lx, m, z, lz, fd, sigma, feat_scale, ell, kappa, a2, b2, h, nsel, sel, nthreads,
                       out, absout, counts, per_target, 1);
}

/*
 * Fourth-order Taylor model of the line G(t) = F(h exp(t xi)) (Sec. VI-B,
 * eq. fourth), xi = (w^, u) in the paper's convention.  Along the line the
 * transformed target moves as z~(t) = exp(-t Xi) z~, so with d = x - z~,
 * u1 = w x z~ + u and u_{k+1} = w x u_k,
 *   x - z~(t) = d + t u1 - t^2/2 u2 + t^3/6 u3 - t^4/24 u4 + O(t^5),
 * and the exponent -|x - z~(t)|^2 / (2 ell^2) = alpha + beta t + gamma t^2
 * + delta t^3 + eps t^4 + O(t^5) with
 *   alpha = -|d|^2/(2 ell^2)           beta  = -<d,u1>/ell^2
 *   gamma = -(|u1|^2 - <d,u2>)/(2 ell^2)
 *   delta =  (<u1,u2> - <d,u3>/3)/(2 ell^2)
 *   eps   = -(|u2|^2/4 + <u1,u3>/3 - <d,u4>/12)/(2 ell^2)
 * (the printed gamma, delta, eps expand |x - (z - t u1 - ... - t^4 u4)|^2
 * instead; the g^1..g^4 compositions below are the paper's).  Then
 *   G(t) ~ F + A1 t + A2 t^2 + A3 t^3 + A4 t^4,
 *   A_k = sigma^2 sum_ij c_ij e^alpha g^k_ij,
 *   g1 = beta, g2 = gamma + beta^2/2, g3 = delta + beta gamma + beta^3/6,
 *   g4 = eps + beta delta + beta^2 gamma/2 + gamma^2/2 + beta^4/24,
 * summed over the pairs inside the cutoff at t = 0.
 * out[5] = F, A1..A4; absout[5] the sums of absolute terms.
 */
typedef struct {
    int n, fd;
    const float *x, *lx, *z, *lz;
    double sigma, sf, ell, kappa;
    double Rt[9], tt[3], w[3], u[3];
    int j0, j1;
    double sum[5], abs_sum[5];
} qjob_t;

static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void* run_qjob(void* arg) {
    qjob_t* J = (qjob_t*)arg;
    const double il2 = 1.0 / (J->ell * J->ell);
    const double rc2 = (J->kappa > 0.0) ? (J->kappa * J->ell) * (J->kappa * J->ell) : INFINITY;
    const double s2 = J->sigma * J->sigma;
    for (int q = 0; q < 5; q++) { J->sum[q] = 0.0; J->abs_sum[q] = 0.0; }
    for (int j = J->j0; j < J->j1; j++) {
        double zt[3], u1[3], u2[3], u3[3], u4[3];
        for (int r = 0; r < 3; r++)
            zt[r] = J->Rt[3 * r] * J->z[3 * j] + J->Rt[3 * r + 1] * J->z[3 * j + 1] +
                    J->Rt[3 * r + 2] * J->z[3 * j + 2] + J->tt[r];
        cross3(J->w, zt, u1);
        for (int r = 0; r < 3; r++) u1[r] += J->u[r];
        cross3(J->w, u1, u2);
        cross3(J->w, u2, u3);
        cross3(J->w, u3, u4);
        for (int i = 0; i < J->n; i++) {
            double d[3];
            for (int r = 0; r < 3; r++) d[r] = (double)J->x[3 * i + r] - zt[r];
            const double r2 = dot3(d, d);
            if (!(r2 <= rc2)) continue;
            double lm = 0.0;
            for (int f = 0; f < J->fd; f++) lm += (double)J->lx[J->fd * i + f] * (double)J->lz[J->fd * j + f];
            const double cw = J->sf * lm * s2 * exp(-0.5 * r2 * il2);
            const double be = -dot3(d, u1) * il2;
            const double ga = -(dot3(u1, u1) - dot3(d, u2)) * 0.5 * il2;
            const double de = (dot3(u1, u2) - dot3(d, u3) / 3.0) * 0.5 * il2;
            const double ep = -(dot3(u2, u2) / 4.0 + dot3(u1, u3) / 3.0 - dot3(d, u4) / 12.0) * 0.5 * il2;
            const double g1 = be;
            const double g2 = ga + be * be / 2.0;
            const double g3 = de + be * ga + be * be * be / 6.0;
            const double g4 = ep + be * de + be * be * ga / 2.0 + ga * ga / 2.0 + be * be * be * be / 24.0;
            const double t5[5] = {cw, cw * g1, cw * g2, cw * g3, cw * g4};
            for (int q = 0; q < 5; q++) { J->sum[q] += t5[q]; J->abs_sum[q] += fabs(t5[q]); }
        }
    }
    return NULL;
}

int cvo_oracle_quartic(int n, const float* x, const float* lx, int m, const float* z, const float* lz,
                       int fd, double sigma, double feat_scale, double ell, double kappa,
                       const double T[16], const double w[3], const double u[3], int nthreads,
                       double out[5], double absout[5]) {
    if (!check_cloud(n, fd, x, lx) || !check_cloud(m, fd, z, lz)) return OR_EINVAL;
    if (!(ell > 0.0) || kappa < 0.0) return OR_EINVAL;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > m) nthreads = m;
    qjob_t* jobs = (qjob_t*)calloc((size_t)nthreads, sizeof(qjob_t));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return OR_EINVAL; }
    double h[16];
    rigid_inverse(T, h);
    for (int k2 = 0; k2 < nthreads; k2++) {
        qjob_t* J = &jobs[k2];
        J->n = n; J->fd = fd; J->x = x; J->lx = lx; J->z = z; J->lz = lz;
        J->sigma = sigma; J->sf = feat_scale; J->ell = ell; J->kappa = kappa;
        pose_to_inverse_action(h, J->Rt, J->tt);
        for (int r = 0; r < 3; r++) { J->w[r] = w[r]; J->u[r] = u[r]; }
        J->j0 = (int)((long long)m * k2 / nthreads);
        J->j1 = (int)((long long)m * (k2 + 1) / nthreads);
    }
    for (int k2 = 1; k2 < nthreads; k2++) pthread_create(&th[k2], NULL, run_qjob, &jobs[k2]);
    run_qjob(&jobs[0]);
    for (int k2 = 1; k2 < nthreads; k2++) pthread_join(th[k2], NULL);
    for (int q = 0; q < 5; q++) { out[q] = 0.0; absout[q] = 0.0; }
    for (int k2 = 0; k2 < nthreads; k2++)
        for (int q = 0; q < 5; q++) { out[q] += jobs[k2].sum[q]; absout[q] += jobs[k2].abs_sum[q]; }
    free(jobs); free(th);
    return OR_OK;
}

/*
 * Step of the quartic model P(t) = A1 t + A2 t^2 + A3 t^3 + A4 t^4 (eq.
 * fourth: the value of t > 0 that maximises the quartic), read as: among the
 * local maxima of P on t > 0 (points where P' = A1 + 2 A2 t + 3 A3 t^2 +
 * 4 A4 t^3 changes sign from + to -), the one with the largest P.  P' is
 * monotone between consecutive roots of P'' (a quadratic), so the real line
 * t > 0 is cut at those roots and at a bound beyond which P' has no root
 * (Cauchy's bound); each piece where P' goes from > 0 to <= 0 holds exactly
 * one such point, found by plain bisection to the last bit.  Returns 1 and
 * *t on success, 0 when P has no local maximum on t > 0 (then the caller
 * falls back).  Coefficients whose size is below 1e-14 of the largest are
 * treated as zero when the degree of P' is decided.
 */
static double poly4(const double A[5], double t) { return t * (A[1] + t * (A[2] + t * (A[3] + t * A[4]))); }
static double dpoly3(const double c[4], double t) { return c[0] + t * (c[1] + t * (c[2] + t * c[3])); }

int cvo_oracle_quartic_step_bounded(const double A[5], double tmax, double* t_out);

int cvo_oracle_quartic_step(const double A[5], double* t_out) {
    return cvo_oracle_quartic_step_bounded(A, INFINITY, t_out);
}

/* The same, counting only the local maxima at t <= tmax: the model is a
 * Taylor expansion of G about t = 0 and is trusted only on (0, tmax]. */
int cvo_oracle_quartic_step_bounded(const double A[5], double tmax, double* t_out) {
    const double c[4] = {A[1], 2.0 * A[2], 3.0 * A[3], 4.0 * A[4]}; /* P' coefficients */
    double big = 0.0;
    for (int i = 0; i < 4; i++) big = fmax(big, fabs(c[i]));
    if (!(big > 0.0) || !isfinite(big)) return 0;
    int deg = 3;
    while (deg > 0 && fabs(c[deg]) <= 1e-14 * big) deg--;
    if (deg == 0) return 0;
    double cc[4] = {c[0], c[1], deg >= 2 ? c[2] : 0.0, deg >= 3 ? c[3] : 0.0};
    double bound = 0.0;
    for (int i = 0; i < deg; i++) bound = fmax(bound, fabs(cc[i] / cc[deg]));
    bound = 1.0 + bound;
    /* cut points: 0, the positive roots of P'' = cc1 + 2 cc2 t + 3 cc3 t^2, bound */
    double cut[4];
    int nc = 0;
    cut[nc++] = 0.0;
    const double qa = 3.0 * cc[3], qb = 2.0 * cc[2], qc = cc[1];
    double r[2];
    int nr = 0;
    if (qa != 0.0) {
        const double disc = qb * qb - 4.0 * qa * qc;
        if (disc > 0.0) {
            r[nr++] = (-qb - sqrt(disc)) / (2.0 * qa);
            r[nr++] = (-qb + sqrt(disc)) / (2.0 * qa);
        }
    } else if (qb != 0.0) {
        r[nr++] = -qc / qb;
    }
    if (nr == 2 && r[0] > r[1]) { const double tmp = r[0]; r[0] = r[1]; r[1] = tmp; }
    for (int i = 0; i < nr; i++)
        if (r[i] > 0.0 && r[i] < bound) cut[nc++] = r[i];
    cut[nc++] = bound;
    int found = 0;
    double best_t = 0.0, best_p = 0.0;
    for (int i = 0; i + 1 < nc; i++) {
        double lo = cut[i], hi = cut[i + 1];
        if (!(dpoly3(cc, lo) > 0.0 && dpoly3(cc, hi) <= 0.0)) continue;
        for (;;) {
            const double mid = lo + 0.5 * (hi - lo);
            if (!(mid > lo && mid < hi)) break;
            if (dpoly3(cc, mid) > 0.0) lo = mid; else hi = mid;
        }
        if (!(hi <= tmax)) continue;
        const double pv = poly4(A, hi);
        if (!found || pv > best_p) { found = 1; best_t = hi; best_p = pv; }
    }
    if (found) *t_out = best_t;
    return found;
}

/*
 * The registration iteration (Section VI): at every iteration k,
 *   ell   = schedule length-scale of the stage containing k
 *   (F, omega, v) at the current h
 *   F <= 1e-300 -> no overlap (error)
 *   xi    = (omega, v) with the components outside dof_mask set to zero (the
 *           flow on the subgroup of SE(3) the mask selects; 0 = all six)
 *   d     = the search direction: xi itself (step rules 0 and 1), or
 *           (step_rule 2, conjugate directions, a project rule) xi + beta d'
 *           with d' the previous iteration's direction and the
 *           Polak-Ribiere beta = max(0, <xi, xi - xi'>_M / <xi', xi'>_M),
 *           xi' the previous iteration's xi and <p, q>_M =
 *           a^2 p_w.q_w + b^2 p_v.q_v the metric of Sec. IV-B; d = xi instead
 *           at the first iteration of each stage, after 6 directions since
 *           the last such restart, and whenever <xi, d>_M <= 0
 *   tau = eta ell^2 / F (step_rule 0), or (step_rules 1, 2) the maximiser of
 *         the quartic model along d when it has one on (0, t_max], else
 *         eta ell^2 / F, with t_max = 3 ell / (|d_w| rho + |d_v|) the step
 *         that moves a typical target by three length-scales (rho = the
 *         targets' root mean square norm + |t_h|): the Taylor model describes
 *         G only near t = 0;
 *   h <- h exp(tau d)
 *   stop when the last stage is reached and |tau d|_2 < tol (the
 *   transformation threshold of Table 1) or |xi|_2 < grad_tol (the
 *   gradient-norm threshold); a zero threshold is off.
 * Stage s spans stage_iters[s] iterations, or ends after the iteration whose
 * applied twist |tau d|_2 < stage_tol (stage_tol > 0); the last stage runs
 * to max_iters.
 * T0 and T_out use the library convention T = h^-1.
 * trace (optional) receives per iteration 26 doubles:
 *   F, omega[3], v[3], tau, ell, within-pairs, then T (16, row-major) after the step;
 * abs_trace (optional) per iteration the 7 sums of |terms| of F, omega, v.
 * use_grid != 0 (with kappa > 0) takes each evaluation's pairs from the grid
 * enumeration (cvo_oracle_eval_grid: the same pair set).
 */
int cvo_oracle_register(int n, const float* x, const float* lx, int m, const float* z, const float* lz,
                        int fd, double sigma, double feat_scale, double a2, double b2, double eta,
                        double kappa, int n_stages, const int* stage_iters, const double* stage_ell,
                        int max_iters, double tol, double grad_tol, int step_rule, int dof_mask,
                        const double T0[16], int nthreads,
                        double T_out[16], double* trace, int* iters_out, int* converged_out,
                        int use_grid, double* abs_trace, double stage_tol) {
    if (n_stages < 1 || !stage_ell || max_iters < 1 || !(eta > 0.0)) return OR_EINVAL;
    if (!(tol >= 0.0) || !(grad_tol >= 0.0) || !(stage_tol >= 0.0)) return OR_EINVAL;
    if (dof_mask < 0 || dof_mask > 63) return OR_EINVAL;
    if (dof_mask == 0) dof_mask = 63;
    for (int s = 0; s < n_stages; s++) {
        if (!(stage_ell[s] > 0.0)) return OR_EINVAL;
        if (s < n_stages - 1 && (!stage_iters || stage_iters[s] < 1)) return OR_EINVAL;
    }
    if (!check_cloud(n, fd, x, lx) || !check_cloud(m, fd, z, lz)) return OR_EINVAL;
    if (!(a2 > 0.0)) a2 = cvo_oracle_mean_sqnorm(n, x);
    /* the targets' root mean square norm */
    const double zrms = sqrt(cvo_oracle_mean_sqnorm(m, z));
    double h[16];
    rigid_inverse(T0, h);
    int stage = 0, stage_start = 0, stage_done = 0, k = 0, conv = 0, rc = OR_OK;
    /* conjugate directions: the previous xi and d, directions since the
       last restart, and the stage they belong to */
    double xi_prev[6] = {0, 0, 0, 0, 0, 0}, d_prev[6] = {0, 0, 0, 0, 0, 0};
    int since_restart = 0, d_stage = -1;
    for (k = 0; k < max_iters; k++) {
        if (stage < n_stages - 1 && (k - stage_start >= stage_iters[stage] || stage_done)) {
            stage_start = k;
            stage++;
        }
        stage_done = 0;
        const double ell = stage_ell[stage];
        double g[7], ga[7];
        long long cnt[2];
        rc = eval_h_impl(n, x, lx, m, z, lz, fd, sigma, feat_scale, ell, kappa, a2, b2, h, 0, NULL, nthreads,
                         g, ga, cnt, NULL, use_grid && kappa > 0.0);
        if (rc != OR_OK) break;
        if (!(g[0] > 1e-300)) { rc = OR_ENOOVERLAP; break; }
        /* the flow on the subgroup dof_mask selects (bits 0-2 omega, 3-5 v):
           the gradient of F restricted to it is the metric-orthogonal
           projection of the full gradient, here the masked components */
        double xi[6];
        for (int q = 0; q < 6; q++) xi[q] = ((dof_mask >> q) & 1) ? g[1 + q] : 0.0;
        double d[6];
        for (int q = 0; q < 6; q++) d[q] = xi[q];
        if (step_rule == 2) {
            int restart = since_restart == 0 || since_restart >= 6 || d_stage != stage;
            if (!restart) {
                double num = 0.0, den = 0.0;
                for (int q = 0; q < 6; q++) {
                    const double wq = q < 3 ? a2 : b2;
                    num += wq * xi[q] * (xi[q] - xi_prev[q]);
                    den += wq * xi_prev[q] * xi_prev[q];
                }
                const double beta = (den > 0.0 && num > 0.0) ? num / den : 0.0;
                double slope = 0.0;
                for (int q = 0; q < 6; q++) {
                    d[q] = xi[q] + beta * d_prev[q];
                    slope += (q < 3 ? a2 : b2) * xi[q] * d[q];
                }
                if (!(slope > 0.0)) restart = 1;
            }
            if (restart) {
                for (int q = 0; q < 6; q++) d[q] = xi[q];
                since_restart = 0;
            }
            since_restart++;
            d_stage = stage;
            for (int q = 0; q < 6; q++) { xi_prev[q] = xi[q]; d_prev[q] = d[q]; }
        }
        double tau = eta * ell * ell / g[0];
        if (step_rule == 1 || step_rule == 2) {
            /* quartic model along d at the current pose, trusted while a
               typical target moves by at most 3 ell: a target moves at
               speed |d_w x z~ + d_v| <= |d_w| |z~| + |d_v|, and the typical
               |z~| is bounded by rho = zrms + |t_h| */
            double Tcur[16], A[5], Aa[5], tq;
            rigid_inverse(h, Tcur);
            rc = cvo_oracle_quartic(n, x, lx, m, z, lz, fd, sigma, feat_scale, ell, kappa, Tcur, d, d + 3,
                                    nthreads, A, Aa);
            if (rc != OR_OK) break;
            const double rho = zrms + sqrt(h[3] * h[3] + h[7] * h[7] + h[11] * h[11]);
            const double speed = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) * rho +
                                 sqrt(d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
            const double tmax = speed > 0.0 ? 3.0 * ell / speed : INFINITY;
            if (cvo_oracle_quartic_step_bounded(A, tmax, &tq)) tau = tq;
        }
        newstep(h, d, d + 3, tau);
        double sq = 0.0, gq = 0.0;
        for (int q = 0; q < 6; q++) {
            sq += (tau * d[q]) * (tau * d[q]);
            gq += xi[q] * xi[q];
        }
        if (trace) {
            double* tr = trace + 26 * (size_t)k;
            for (int q = 0; q < 7; q++) tr[q] = g[q];
            tr[7] = tau; tr[8] = ell; tr[9] = (double)cnt[0];
            rigid_inverse(h, tr + 10);
        }
        if (abs_trace)
            for (int q = 0; q < 7; q++) abs_trace[7 * (size_t)k + q] = ga[q];
        if (stage == n_stages - 1 && (sqrt(sq) < tol || sqrt(gq) < grad_tol)) { conv = 1; k++; break; }
        /* a stage also ends once its own applied twist is below stage_tol */
        stage_done = sqrt(sq) < stage_tol;
    }
    rigid_inverse(h, T_out);
    if (iters_out) *iters_out = k;
    if (converged_out) *converged_out = conv;
    return rc;
}
