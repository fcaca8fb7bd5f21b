/*
 * Stein ICP oracle: a plain, slow, obviously correct CPU implementation of
 * one Stein-ICP iteration, written from the paper
 *   F. Afzal Maken, F. Ramos, L. Ott, "Stein ICP for Uncertainty Estimation
 *   in Point Cloud Matching", arXiv:2106.03287.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file. It shares no code, header,
 * table or helper with the HIP library; the product path never calls it.
 *
 * Precision: FP64 throughout, with one exception fixed by the precision rule
 * for decisions: the nearest-neighbour argmin (Eq. 1) decides an integer, so
 * it is taken in the kernel's precision, FP32, on the FP64 transformed point
 * rounded once to FP32, with the squared distance formed as
 *   dx = qx - rx, dy = qy - ry, dz = qz - rz  (FP32)
 *   d  = fma(dz, dz, fma(dy, dy, dx * dx))     (FP32, fused multiply-adds)
 * and ties broken towards the lowest reference index. Everything else
 * (residuals, gradients, kernels, bandwidths, optimiser) is FP64.
 *
 * Build with -ffp-contract=off: every a*b+c below is two rounded operations
 * unless written as fma()/fmaf().
 *
 * Readings of points the paper leaves open (each is a documented choice):
 *  - Gradient scale: the mean minibatch gradient of Eqs. 4-5 as printed,
 *    i.e. the gradient of E_m = (1/2m) sum ||e||^2 (no factor 2).
 *  - Eq. 16 sums without 1/K; Eq. 11 is an expectation, so phi is averaged
 *    over the K particles (divided by K).
 *  - Posterior score: G = -N gbar + grad log prior, N = full source size.
 *  - The repulsive term differentiates the kernel with respect to the
 *    summed particle theta_l (Eq. 13), which makes it repulsive.
 *  - Rotation kernel (Eq. 17): sum over the three angles of the squared
 *    wrapped difference atan2(sin d, cos d); translation and rotation have
 *    separate kernels and bandwidths.
 *  - Median heuristic: h = med^2 / ln K, med = median of the K(K-1)/2
 *    distances between distinct particles (mean of the two middle values
 *    for an even count); K = 1 or med = 0 gives h = 1.
 *  - Euler convention: R = Rz(yaw) Ry(pitch) Rx(roll); the state is not
 *    wrapped.
 *  - Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step count
 *    from 1) is applied to the descent direction -phi.
 *  - Prior (Eqs. 14-15): Gaussian translation prior with variance sigma
 *    (Eq. 14 divides by it), von Mises rotation prior with concentration
 *    kappa; uniform (zero gradient) by default, as in the experiments.
 *  - Point-to-plane metric (used for the paper's quantitative results,
 *    Sec. V, and cited to Chen and Medioni in Sec. II without a formula):
 *    matches still by Eq. 1; the residual of a matched pair is its
 *    projection rho = n^T e onto the unit normal n of the matched reference
 *    point; the cost is E_m = (1/2m) sum rho^2 (the scale of the
 *    point-to-point reading above). Normals: eigenvector of the smallest
 *    eigenvalue of the covariance of the point's k nearest references (the
 *    point itself included, neighbours decided in FP32 like Eq. 1); zero
 *    where that eigenvalue is not separated from the middle one by more
 *    than 1e-10 of the trace (a line, a point or an isotropic
 *    neighbourhood: no unique plane). The sign of a normal is left open:
 *    neither the cost nor its gradient depends on it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t K;              /* number of particles */
    int32_t m;              /* minibatch size */
    int64_t N;              /* source size, scales the mean gradient (Eq. 16) */
    int64_t M;              /* reference size */
    double lr, beta1, beta2, eps;
    int32_t optimizer;      /* 0: Adam on -phi; 1: theta += lr * phi (Eq. 12) */
    int32_t bandwidth;      /* 0: median heuristic; 1: fixed h */
    double h_fixed_trans, h_fixed_rot;
    int32_t prior;          /* 0: uniform; 1: Gaussian + von Mises (Eqs. 14-15) */
    int32_t pad_;
    double prior_mu[6];
    double prior_var_trans[3];
    double prior_kappa_rot[3];
    int32_t metric;         /* 0: point-to-point (Eqs. 4-5); 1: point-to-plane */
    int32_t pad2_;
} or_config;

/* ---------------------------------------------------------------------- */
/* 3x3 helpers (row-major)                                                */
/* ---------------------------------------------------------------------- */

static void mat3_mul(const double A[9], const double B[9], double C[9])
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            C[3 * r + c] = (A[3 * r + 0] * B[0 + c] + A[3 * r + 1] * B[3 + c]) + A[3 * r + 2] * B[6 + c];
}

static void mat3_mul3(const double A[9], const double B[9], const double C[9], double D[9])
{
    double AB[9];
    mat3_mul(A, B, AB);
    mat3_mul(AB, C, D);
}

/* ---------------------------------------------------------------------- */
/* Pose -> rotation and its partial derivatives.                          */
/* theta = (x, y, z, roll, pitch, yaw); R parametrised by theta_4:6 (Sec.  */
/* III-A), R = Rz(yaw) Ry(pitch) Rx(roll). dR holds dR/droll, dR/dpitch,   */
/* dR/dyaw (three row-major 3x3 blocks), the factors of Eq. 5.            */
/* ---------------------------------------------------------------------- */
void or_rotation(const double th[6], double R[9], double dR[27])
{
    const double cr = cos(th[3]), sr = sin(th[3]);
    const double cp = cos(th[4]), sp = sin(th[4]);
    const double cy = cos(th[5]), sy = sin(th[5]);
    const double Rx[9]  = {1, 0, 0, 0, cr, -sr, 0, sr, cr};
    const double Ry[9]  = {cp, 0, sp, 0, 1, 0, -sp, 0, cp};
    const double Rz[9]  = {cy, -sy, 0, sy, cy, 0, 0, 0, 1};
    const double dRx[9] = {0, 0, 0, 0, -sr, -cr, 0, cr, -sr};
    const double dRy[9] = {-sp, 0, cp, 0, 0, 0, -cp, 0, -sp};
    const double dRz[9] = {-sy, -cy, 0, cy, -sy, 0, 0, 0, 0};
    mat3_mul3(Rz, Ry, Rx, R);
    if (dR) {
        mat3_mul3(Rz, Ry, dRx, dR + 0);
        mat3_mul3(Rz, dRy, Rx, dR + 9);
        mat3_mul3(dRz, Ry, Rx, dR + 18);
    }
}

/* s' = R s + u (Eq. 1), FP64, each product and sum rounded separately. */
void or_transform(const double R[9], const double u[3], const float s[3], double q[3])
{
    const double s0 = s[0], s1 = s[1], s2 = s[2];
    for (int r = 0; r < 3; ++r)
        q[r] = ((R[3 * r + 0] * s0 + R[3 * r + 1] * s1) + R[3 * r + 2] * s2) + u[r];
}

/* Squared Euclidean distance in FP32 (the precision the argmin is decided in). */
float or_dist2_f32(const float q[3], const float r[3])
{
    const float dx = q[0] - r[0];
    const float dy = q[1] - r[1];
    const float dz = q[2] - r[2];
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

/* Eq. 1 by exhaustive scan: for each query the reference index with the
 * smallest squared distance; ties go to the lowest index. */
void or_nn_f32(const float *q, int64_t nq, const float *ref, int64_t M,
               int32_t *idx, float *d2)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nq; ++i) {
        float best = INFINITY;
        int32_t bi = -1;
        for (int64_t j = 0; j < M; ++j) {
            const float d = or_dist2_f32(q + 3 * i, ref + 3 * j);
            if (d < best) {
                best = d;
                bi = (int32_t)j;
            }
        }
        idx[i] = bi;
        if (d2) d2[i] = best;
    }
}

/* Minibatch cost E_m(theta) = (1/2m) sum_i ||R s_i + u - r_match(i)||^2
 * (Eq. 2 over the minibatch, scaled so that its gradient is Eqs. 4-5). */
double or_icp_cost(const double th[6], const float *src, const float *ref,
                   const int32_t *batch, int32_t m, const int32_t *match)
{
    double R[9], q[3];
    or_rotation(th, R, NULL);
    double acc = 0.0;
    for (int32_t i = 0; i < m; ++i) {
        or_transform(R, th, src + 3 * (int64_t)batch[i], q);
        const float *r = ref + 3 * (int64_t)match[i];
        const double e0 = q[0] - r[0], e1 = q[1] - r[1], e2 = q[2] - r[2];
        acc += (e0 * e0 + e1 * e1) + e2 * e2;
    }
    return acc / (2.0 * m);
}

/* Mean minibatch gradient, Eqs. 4-5: translation part (1/m) sum e_i,
 * rotation part (1/m) sum e_i^T (dR/dtheta_d) s_i, with e_i = R s_i + u - r. */
void or_icp_gradient(const double th[6], const float *src, const float *ref,
                     const int32_t *batch, int32_t m, const int32_t *match, double g[6])
{
    double R[9], dR[27], q[3];
    or_rotation(th, R, dR);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int32_t i = 0; i < m; ++i) {
        const float *s = src + 3 * (int64_t)batch[i];
        or_transform(R, th, s, q);
        const float *r = ref + 3 * (int64_t)match[i];
        const double e[3] = {q[0] - r[0], q[1] - r[1], q[2] - r[2]};
        acc[0] += e[0];
        acc[1] += e[1];
        acc[2] += e[2];
        for (int d = 0; d < 3; ++d) {
            const double *D = dR + 9 * d;
            double v[3];
            for (int row = 0; row < 3; ++row)
                v[row] = (D[3 * row + 0] * s[0] + D[3 * row + 1] * s[1]) + D[3 * row + 2] * s[2];
            acc[3 + d] += (e[0] * v[0] + e[1] * v[1]) + e[2] * v[2];
        }
    }
    for (int d = 0; d < 6; ++d) g[d] = acc[d] / m;
}

/* Gradient of the log prior: Eq. 14 (translation) and Eq. 15 (rotation). */
void or_prior_grad(const or_config *c, const double th[6], double out[6])
{
    for (int d = 0; d < 6; ++d) out[d] = 0.0;
    if (c->prior != 1) return;
    for (int d = 0; d < 3; ++d)
        out[d] = -(th[d] - c->prior_mu[d]) / c->prior_var_trans[d];
    for (int d = 0; d < 3; ++d)
        out[3 + d] = -c->prior_kappa_rot[d] * sin(th[3 + d] - c->prior_mu[3 + d]);
}

/* ---------------------------------------------------------------------- */
/* Point-to-plane metric                                                   */
/* ---------------------------------------------------------------------- */

/* The k nearest references of each query under Eq. 1's metric, decided in
 * FP32 like the argmin: the k smallest (distance, index) pairs in ascending
 * order, ties to the lower index. Slots beyond M hold index -1 and an
 * infinite distance. Plain insertion into a sorted list of k. */
void or_knn_f32(const float *q, int64_t nq, const float *ref, int64_t M, int32_t k,
                int32_t *idx, float *d2)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nq; ++i) {
        int32_t *bi = idx + i * k;
        float *bd = d2 + i * k;
        for (int32_t s = 0; s < k; ++s) {
            bi[s] = -1;
            bd[s] = INFINITY;
        }
        for (int64_t j = 0; j < M; ++j) {
            const float d = or_dist2_f32(q + 3 * i, ref + 3 * j);
            if (!(d < bd[k - 1])) continue;   /* equal distance: the lower index stays */
            int32_t s = k - 1;
            while (s > 0 && d < bd[s - 1]) {
                bd[s] = bd[s - 1];
                bi[s] = bi[s - 1];
                --s;
            }
            bd[s] = d;
            bi[s] = (int32_t)j;
        }
    }
}

/* Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations:
 * each rotation in the (p, q) plane zeroes A[p][q]; sweeps repeat until the
 * off-diagonal part vanishes at FP64 precision. Eigenvalues w ascending,
 * eigenvector i in column i of V (row-major). */
static void jacobi_eigen3(const double A_in[9], double w[3], double V[9])
{
    double A[3][3], U[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            A[r][c] = A_in[3 * r + c];
            U[r][c] = r == c ? 1.0 : 0.0;
        }
    static const int PQ[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int sweep = 0; sweep < 64; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off == 0.0 || off <= 1e-36 * dia) break;
        for (int e = 0; e < 3; ++e) {
            const int p = PQ[e][0], qq = PQ[e][1];
            const double apq = A[p][qq];
            if (apq == 0.0) continue;
            const double th = (A[qq][qq] - A[p][p]) / (2.0 * apq);
            double t;
            if (fabs(th) > 1e150)
                t = 0.5 / th;
            else
                t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
            /* A <- J^T A J with J the rotation by (c, sn) in the (p, q) plane */
            for (int r = 0; r < 3; ++r) {
                const double arp = A[r][p], arq = A[r][qq];
                A[r][p] = c * arp - sn * arq;
                A[r][qq] = sn * arp + c * arq;
            }
            for (int r = 0; r < 3; ++r) {
                const double apr = A[p][r], aqr = A[qq][r];
                A[p][r] = c * apr - sn * aqr;
                A[qq][r] = sn * apr + c * aqr;
            }
            A[p][qq] = A[qq][p] = 0.0;
            for (int r = 0; r < 3; ++r) {
                const double urp = U[r][p], urq = U[r][qq];
                U[r][p] = c * urp - sn * urq;
                U[r][qq] = sn * urp + c * urq;
            }
        }
    }
    int order[3] = {0, 1, 2};
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (A[order[b]][order[b]] < A[order[a]][order[a]]) {
                const int tmp = order[a];
                order[a] = order[b];
                order[b] = tmp;
            }
    for (int i = 0; i < 3; ++i) {
        w[i] = A[order[i]][order[i]];
        for (int r = 0; r < 3; ++r) V[3 * r + i] = U[r][order[i]];
    }
}

/* Unit normal of every reference point from its k nearest references (the
 * point itself included; all M when M < k): the covariance
 * (1/k) sum (p - mean)(p - mean)^T in FP64 and its eigenvector of the
 * smallest eigenvalue; zero when the smallest and middle eigenvalues are
 * within 1e-10 of the trace of each other (no unique plane). normals: M x 3; eig
 * (optional): M x 3 eigenvalues, ascending. */
void or_normals(const float *ref, int64_t M, int32_t k, double *normals, double *eig)
{
    const int32_t kk = (int64_t)k < M ? k : (int32_t)M;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)M * kk);
    float *d2 = (float *)malloc(sizeof(float) * (size_t)M * kk);
    or_knn_f32(ref, M, ref, M, kk, idx, d2);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        const int32_t *nb = idx + i * kk;
        double mu[3] = {0, 0, 0};
        for (int32_t s = 0; s < kk; ++s)
            for (int d = 0; d < 3; ++d) mu[d] += ref[3 * (int64_t)nb[s] + d];
        for (int d = 0; d < 3; ++d) mu[d] /= kk;
        double C[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int32_t s = 0; s < kk; ++s) {
            double v[3];
            for (int d = 0; d < 3; ++d) v[d] = ref[3 * (int64_t)nb[s] + d] - mu[d];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) C[3 * r + c] += v[r] * v[c];
        }
        for (int e = 0; e < 9; ++e) C[e] /= kk;
        double w[3], V[9];
        jacobi_eigen3(C, w, V);
        double n[3] = {V[0], V[3], V[6]};
        const double trace = (w[0] + w[1]) + w[2];
        if (w[1] - w[0] > 1e-10 * trace) {
            const double len = sqrt((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
            for (int d = 0; d < 3; ++d) n[d] /= len;
        } else {
            n[0] = n[1] = n[2] = 0.0;
        }
        for (int d = 0; d < 3; ++d) normals[3 * i + d] = n[d];
        if (eig)
            for (int d = 0; d < 3; ++d) eig[3 * i + d] = w[d];
    }
    free(idx);
    free(d2);
}

/* Point-to-plane minibatch cost E_m = (1/2m) sum_i (n_j^T e_i)^2, with
 * j = match(i) and e_i = R s_i + u - r_j. */
double or_plane_cost(const double th[6], const float *src, const float *ref, const double *normals,
                     const int32_t *batch, int32_t m, const int32_t *match)
{
    double R[9], q[3];
    or_rotation(th, R, NULL);
    double acc = 0.0;
    for (int32_t i = 0; i < m; ++i) {
        or_transform(R, th, src + 3 * (int64_t)batch[i], q);
        const float *r = ref + 3 * (int64_t)match[i];
        const double *n = normals + 3 * (int64_t)match[i];
        const double rho = (n[0] * (q[0] - r[0]) + n[1] * (q[1] - r[1])) + n[2] * (q[2] - r[2]);
        acc += rho * rho;
    }
    return acc / (2.0 * m);
}

/* Its gradient: translation part (1/m) sum rho_i n_j, rotation part
 * (1/m) sum rho_i n_j^T (dR/dtheta_d) s_i (Eq. 5 with e projected on n). */
void or_plane_gradient(const double th[6], const float *src, const float *ref, const double *normals,
                       const int32_t *batch, int32_t m, const int32_t *match, double g[6])
{
    double R[9], dR[27], q[3];
    or_rotation(th, R, dR);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int32_t i = 0; i < m; ++i) {
        const float *s = src + 3 * (int64_t)batch[i];
        or_transform(R, th, s, q);
        const float *r = ref + 3 * (int64_t)match[i];
        const double *n = normals + 3 * (int64_t)match[i];
        const double e[3] = {q[0] - r[0], q[1] - r[1], q[2] - r[2]};
        const double rho = (n[0] * e[0] + n[1] * e[1]) + n[2] * e[2];
        for (int d = 0; d < 3; ++d) acc[d] += rho * n[d];
        for (int d = 0; d < 3; ++d) {
            const double *D = dR + 9 * d;
            double v[3];
            for (int row = 0; row < 3; ++row)
                v[row] = (D[3 * row + 0] * s[0] + D[3 * row + 1] * s[1]) + D[3 * row + 2] * s[2];
            acc[3 + d] += rho * ((n[0] * v[0] + n[1] * v[1]) + n[2] * v[2]);
        }
    }
    for (int d = 0; d < 6; ++d) g[d] = acc[d] / m;
}

/* Wrapped angle difference used by the rotation kernel (Eq. 17). */
static double wrap_angle(double x) { return atan2(sin(x), cos(x)); }

static int cmp_double(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Median of n values (a library sort, then the middle one, or the mean of
 * the two middle ones for even n). */
double or_median(const double *vals, int64_t n)
{
    if (n <= 0) return 0.0;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(tmp, vals, sizeof(double) * (size_t)n);
    qsort(tmp, (size_t)n, sizeof(double), cmp_double);
    const double med = (n % 2) ? tmp[n / 2] : 0.5 * (tmp[n / 2 - 1] + tmp[n / 2]);
    free(tmp);
    return med;
}

/* Median-heuristic bandwidth h = med^2 / ln K over the distances between
 * distinct particles; dist2 is the K x K matrix of squared distances. */
static double median_bandwidth(int K, const double *dist2)
{
    if (K < 2) return 1.0;
    const int64_t P = (int64_t)K * (K - 1) / 2;
    double *d = (double *)malloc(sizeof(double) * (size_t)P);
    int64_t p = 0;
    for (int k = 0; k < K; ++k)
        for (int l = k + 1; l < K; ++l)
            d[p++] = sqrt(dist2[(int64_t)k * K + l]);
    const double med = or_median(d, P);
    free(d);
    if (!(med > 0.0)) return 1.0;
    return (med * med) / log((double)K);
}

/* Stein-ICP direction, Eq. 16 with the kernels of the paper's Sec. IV:
 * translation kernel exp(-||dt||^2 / h_t), rotation kernel (Eq. 17)
 * exp(-sum_d wrap(dr_d)^2 / h_r). For each particle k,
 *   phi_k = (1/K) sum_l [ G_l k(theta_l, theta_k) + grad_{theta_l} k(theta_l, theta_k) ]
 * evaluated separately for theta_1:3 and theta_4:6. h[0], h[1] receive the
 * bandwidths used. */
void or_svgd_phi(const or_config *c, const double *theta, const double *G,
                 double *phi, double h[2])
{
    const int K = c->K;
    double *Dt = (double *)malloc(sizeof(double) * (size_t)K * K);
    double *Dr = (double *)malloc(sizeof(double) * (size_t)K * K);
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l) {
            const double *a = theta + 6 * (int64_t)k, *b = theta + 6 * (int64_t)l;
            double st = 0.0, sr = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double dt = a[d] - b[d];
                st += dt * dt;
                const double dr = wrap_angle(a[3 + d] - b[3 + d]);
                sr += dr * dr;
            }
            Dt[(int64_t)k * K + l] = st;
            Dr[(int64_t)k * K + l] = sr;
        }
    double ht, hr;
    if (c->bandwidth == 1) {
        ht = c->h_fixed_trans;
        hr = c->h_fixed_rot;
    } else {
        ht = median_bandwidth(K, Dt);
        hr = median_bandwidth(K, Dr);
    }
    for (int k = 0; k < K; ++k) {
        const double *tk = theta + 6 * (int64_t)k;
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int l = 0; l < K; ++l) {
            const double *tl = theta + 6 * (int64_t)l;
            const double kt = exp(-Dt[(int64_t)l * K + k] / ht);
            const double kr = exp(-Dr[(int64_t)l * K + k] / hr);
            for (int d = 0; d < 3; ++d) {
                /* grad wrt theta_l of exp(-||theta_l - theta_k||^2 / h) */
                const double rep_t = -(2.0 / ht) * (tl[d] - tk[d]) * kt;
                acc[d] += G[6 * (int64_t)l + d] * kt + rep_t;
                const double rep_r = -(2.0 / hr) * wrap_angle(tl[3 + d] - tk[3 + d]) * kr;
                acc[3 + d] += G[6 * (int64_t)l + 3 + d] * kr + rep_r;
            }
        }
        for (int d = 0; d < 6; ++d) phi[6 * (int64_t)k + d] = acc[d] / K;
    }
    if (h) {
        h[0] = ht;
        h[1] = hr;
    }
    free(Dt);
    free(Dr);
}

/* Update of all particles: Eq. 12 as an ascent along phi, with Adam (the
 * optimiser the experiments use) applied to the descent direction -phi.
 * t is the step count after this update (1 for the first). */
void or_update(const or_config *c, int64_t t, double *theta, double *mom, double *vel,
               const double *phi)
{
    const int64_t n = 6 * (int64_t)c->K;
    if (c->optimizer == 1) {
        for (int64_t i = 0; i < n; ++i) theta[i] += c->lr * phi[i];
        return;
    }
    const double bc1 = 1.0 - pow(c->beta1, (double)t);
    const double bc2 = 1.0 - pow(c->beta2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        const double g = -phi[i];
        mom[i] = c->beta1 * mom[i] + (1.0 - c->beta1) * g;
        vel[i] = c->beta2 * vel[i] + (1.0 - c->beta2) * (g * g);
        const double mhat = mom[i] / bc1;
        const double vhat = vel[i] / bc2;
        theta[i] -= c->lr * mhat / (sqrt(vhat) + c->eps);
    }
}

/* One Stein-ICP iteration (Sec. IV, closing procedure): transform the
 * minibatch by every particle, match each transformed point (Eq. 1), mean
 * gradients per particle (Eqs. 4-5), Stein direction (Eq. 16), update.
 * *t counts completed updates and is advanced by one. Optional outputs (may
 * be NULL): gbar K x 6, phi K x 6, h[2], match K x m. normals (M x 3) is
 * read only with the point-to-plane metric. */
void or_step(const or_config *c, const float *src, const float *ref, const double *normals,
             const int32_t *batch, double *theta, double *mom, double *vel, int64_t *t,
             double *gbar_out, double *phi_out, double *h_out, int32_t *match_out)
{
    const int K = c->K, m = c->m;
    const int64_t nq = (int64_t)K * m;
    float *q32 = (float *)malloc(sizeof(float) * 3 * (size_t)nq);
    int32_t *match = (int32_t *)malloc(sizeof(int32_t) * (size_t)nq);
    double *gbar = (double *)malloc(sizeof(double) * 6 * (size_t)K);
    double *G = (double *)malloc(sizeof(double) * 6 * (size_t)K);
    double *phi = (double *)malloc(sizeof(double) * 6 * (size_t)K);

    for (int k = 0; k < K; ++k) {
        double R[9], q[3];
        or_rotation(theta + 6 * (int64_t)k, R, NULL);
        for (int i = 0; i < m; ++i) {
            or_transform(R, theta + 6 * (int64_t)k, src + 3 * (int64_t)batch[i], q);
            for (int d = 0; d < 3; ++d) q32[3 * ((int64_t)k * m + i) + d] = (float)q[d];
        }
    }
    or_nn_f32(q32, nq, ref, c->M, match, NULL);
    for (int k = 0; k < K; ++k) {
        double pg[6];
        if (c->metric == 1)
            or_plane_gradient(theta + 6 * (int64_t)k, src, ref, normals, batch, m, match + (int64_t)k * m,
                              gbar + 6 * (int64_t)k);
        else
            or_icp_gradient(theta + 6 * (int64_t)k, src, ref, batch, m, match + (int64_t)k * m,
                            gbar + 6 * (int64_t)k);
        or_prior_grad(c, theta + 6 * (int64_t)k, pg);
        for (int d = 0; d < 6; ++d)
            G[6 * (int64_t)k + d] = -(double)c->N * gbar[6 * (int64_t)k + d] + pg[d];
    }
    double h[2];
    or_svgd_phi(c, theta, G, phi, h);
    *t += 1;
    or_update(c, *t, theta, mom, vel, phi);

    if (gbar_out) memcpy(gbar_out, gbar, sizeof(double) * 6 * (size_t)K);
    if (phi_out) memcpy(phi_out, phi, sizeof(double) * 6 * (size_t)K);
    if (h_out) memcpy(h_out, h, sizeof(h));
    if (match_out) memcpy(match_out, match, sizeof(int32_t) * (size_t)nq);
    free(q32);
    free(match);
    free(gbar);
    free(G);
    free(phi);
}

/* T iterations; iteration with step count t uses schedule row t mod rows. */
void or_run(const or_config *c, const float *src, const float *ref, const double *normals,
            const int32_t *schedule, int32_t rows, int32_t T,
            double *theta, double *mom, double *vel, int64_t *t)
{
    for (int32_t it = 0; it < T; ++it) {
        const int32_t *batch = schedule + (int64_t)(*t % rows) * c->m;
        or_step(c, src, ref, normals, batch, theta, mom, vel, t, NULL, NULL, NULL, NULL);
    }
}
