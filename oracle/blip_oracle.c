/*
 * FP64 CPU oracle for blip (periodic cubic B-spline) orbital evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it.  It
 * shares no code, header or constant table with the HIP library.
 *
 * What it computes (Sec. II.B "Orbital evaluation"):
 *   psi_l(r_j) = sum_{s=1..64} a_{l,s} Theta_s(r_j)              Eq. (11.12.24.1)
 *   Theta_s(r) = phi((x-X_s)/b_x) phi((y-Y_s)/b_y) phi((z-Z_s)/b_z)   Eq. (11.12.24.2)
 * where s runs over the 4x4x4 sites of the periodic grid whose basis
 * function is non-zero at r (the subset of Eq. (7)), and phi is the
 * normalised uniform cubic B-spline.  The paper calls phi a "second order
 * polynomial" while giving it a four-site support per direction; the reading
 * taken here is the piecewise cubic with support (-2, 2) and unit sum over
 * the integers.
 *
 * Geometry for a general cell: lattice rows a_1, a_2, a_3 (bohr).  Grid site
 * (i_1, i_2, i_3) sits at sum_d (i_d / n_d) a_d.  A position r has
 * fractional coordinate u = r A^{-1}; grid coordinate t_d = n_d u_d, so
 * Theta_s(r) = prod_d phi(t_d - i_d(s)), which for an orthorhombic cell is
 * exactly Eq. (11.12.24.2) with b_d = |a_d| / n_d.
 *
 * Derivatives (the gradient and Laplacian the local energy needs):
 *   d t_d / d r_c = n_d G_{cd} =: M_{cd}   with G = A^{-1},
 *   grad_c psi = sum_d M_{cd} d psi / d t_d,
 *   lap psi    = sum_{d,e} g_{de} d^2 psi / (d t_d d t_e),  g_{de} = sum_c M_{cd} M_{ce}.
 *
 * Complex orbitals at a k-point: the expansion gives the lattice-periodic
 * part u_l; psi_l = exp(i k.r) u_l with the caller's unwrapped r, so
 *   grad psi = exp(i k.r) (grad u + i k u),
 *   lap psi  = exp(i k.r) (lap u + 2 i k.grad u - |k|^2 u).
 *
 * Non-finite positions give NaN outputs for that position.
 *
 * Arithmetic is FP64 throughout and is compiled without FMA contraction so
 * that the wrap and the cell-index decision are reproducible.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Coefficient storage kinds accepted by oracle_eval. */
enum { ORC_F64 = 0, ORC_F32 = 1, ORC_C128 = 2, ORC_C64 = 3 };

/* ---------------------------------------------------------------------- */
/* The 1-D basis function phi and its first two derivatives, by cases of |x|.
 *   phi(x) = 2/3 - x^2 + |x|^3 / 2     for |x| < 1
 *          = (2 - |x|)^3 / 6           for 1 <= |x| < 2
 *          = 0                         otherwise                          */
double oracle_phi(double x)
{
    double ax = fabs(x);
    if (ax < 1.0) return 2.0 / 3.0 - ax * ax + 0.5 * ax * ax * ax;
    if (ax < 2.0) { double q = 2.0 - ax; return q * q * q / 6.0; }
    return 0.0;
}

double oracle_dphi(double x)
{
    double ax = fabs(x);
    double sg = (x < 0.0) ? -1.0 : 1.0;
    if (ax < 1.0) return sg * (-2.0 * ax + 1.5 * ax * ax);
    if (ax < 2.0) { double q = 2.0 - ax; return -sg * 0.5 * q * q; }
    return 0.0;
}

double oracle_d2phi(double x)
{
    double ax = fabs(x);
    if (ax < 1.0) return -2.0 + 3.0 * ax;
    if (ax < 2.0) return 2.0 - ax;
    return 0.0;
}

/* ---------------------------------------------------------------------- */
/* G = A^{-1} by explicit cofactors.  A is row-major with rows a_1, a_2, a_3.
 * Returns 0 on success, -1 if A is singular or not finite.              */
int oracle_inverse3(const double A[9], double G[9])
{
    double c00 = A[4] * A[8] - A[5] * A[7];
    double c01 = A[5] * A[6] - A[3] * A[8];
    double c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    if (!(fabs(det) > 0.0) || !isfinite(det)) return -1;
    /* inverse = adjugate / det; adjugate is the transposed cofactor matrix */
    G[0] = c00 / det;
    G[3] = c01 / det;
    G[6] = c02 / det;
    G[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    G[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    G[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    G[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    G[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    G[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Selection of the site subset (Eq. (7)): wrap r into the cell and split the
 * grid coordinate into the cell index i0 and the offset f in [0, 1).
 *   u_d = sum_c r_c G_{cd};  u_d <- u_d - floor(u_d)  (a result of 1.0 -> 0.0)
 *   t_d = u_d n_d;  i0_d = floor(t_d)  (i0_d == n_d -> 0);  f_d = t_d - i0_d
 * Returns 0, or -1 for a non-finite position (i0 = 0, f = NaN then).     */
int oracle_wrap(const double G[9], const int n[3], const double r[3],
                int i0[3], double f[3])
{
    int d, bad = 0;
    for (d = 0; d < 3; ++d) {
        double u = r[0] * G[0 * 3 + d];
        u = u + r[1] * G[1 * 3 + d];
        u = u + r[2] * G[2 * 3 + d];
        if (!isfinite(u)) { bad = 1; i0[d] = 0; f[d] = NAN; continue; }
        u = u - floor(u);
        if (u >= 1.0) u = 0.0;
        double t = u * (double)n[d];
        double fl = floor(t);
        int i = (int)fl;
        double fr = t - fl;
        if (i >= n[d]) { i = 0; fr = 0.0; }
        i0[d] = i;
        f[d] = fr;
    }
    return bad ? -1 : 0;
}

static int pmod(int i, int n) { int m = i % n; return m < 0 ? m + n : m; }

static double coef_re(const void* a, int kind, int64_t idx)
{
    switch (kind) {
    case ORC_F64: return ((const double*)a)[idx];
    case ORC_F32: return (double)((const float*)a)[idx];
    case ORC_C128: return ((const double*)a)[2 * idx];
    default: return (double)((const float*)a)[2 * idx];
    }
}

static double coef_im(const void* a, int kind, int64_t idx)
{
    switch (kind) {
    case ORC_C128: return ((const double*)a)[2 * idx + 1];
    case ORC_C64: return (double)((const float*)a)[2 * idx + 1];
    default: return 0.0;
    }
}

/* ---------------------------------------------------------------------- */
/* One position: accumulate psi_l, grad psi_l, lap psi_l for every orbital l.
 * val/grad/lap point at this position's output rows; complex outputs are
 * interleaved (re, im).                                                   */
static void eval_one(const double G[9], const double M[9], const double g[9],
                     const int n[3], int L, const void* a, int kind,
                     const double* kvec, const double r[3],
                     double* val, double* grad, double* lap)
{
    const int cplx = (kind == ORC_C128 || kind == ORC_C64);
    const int w = cplx ? 2 : 1;
    int i0[3];
    double f[3];
    int l, c, d, e;

    if (val) memset(val, 0, sizeof(double) * (size_t)w * L);
    if (grad) memset(grad, 0, sizeof(double) * (size_t)w * 3 * L);
    if (lap) memset(lap, 0, sizeof(double) * (size_t)w * L);

    if (oracle_wrap(G, n, r, i0, f) != 0) {
        for (l = 0; l < w * L; ++l) {
            if (val) val[l] = NAN;
            if (lap) lap[l] = NAN;
        }
        if (grad) for (l = 0; l < w * 3 * L; ++l) grad[l] = NAN;
        return;
    }

    /* The 64 sites s of the subset: i_d = i0_d - 1 + m_d, m_d = 0..3.
     * For each, Theta_s and its derivatives in grid coordinates t.       */
    int m1, m2, m3;
    for (m1 = 0; m1 < 4; ++m1)
    for (m2 = 0; m2 < 4; ++m2)
    for (m3 = 0; m3 < 4; ++m3) {
        int m[3] = {m1, m2, m3};
        double p[3], dp[3], d2p[3];
        for (d = 0; d < 3; ++d) {
            /* t_d - i_d with i_d = i0_d - 1 + m_d */
            double x = f[d] + 1.0 - (double)m[d];
            p[d] = oracle_phi(x);
            dp[d] = oracle_dphi(x);
            d2p[d] = oracle_d2phi(x);
        }
        double theta = p[0] * p[1] * p[2];
        double dt[3];             /* d Theta / d t_d */
        dt[0] = dp[0] * p[1] * p[2];
        dt[1] = p[0] * dp[1] * p[2];
        dt[2] = p[0] * p[1] * dp[2];
        double h[9];              /* d^2 Theta / d t_d d t_e */
        h[0] = d2p[0] * p[1] * p[2];
        h[4] = p[0] * d2p[1] * p[2];
        h[8] = p[0] * p[1] * d2p[2];
        h[1] = h[3] = dp[0] * dp[1] * p[2];
        h[2] = h[6] = dp[0] * p[1] * dp[2];
        h[5] = h[7] = p[0] * dp[1] * dp[2];
        double gth[3];            /* Cartesian gradient of Theta_s */
        for (c = 0; c < 3; ++c) {
            gth[c] = 0.0;
            for (d = 0; d < 3; ++d) gth[c] += M[c * 3 + d] * dt[d];
        }
        double lth = 0.0;         /* Cartesian Laplacian of Theta_s */
        for (d = 0; d < 3; ++d)
            for (e = 0; e < 3; ++e) lth += g[d * 3 + e] * h[d * 3 + e];

        int64_t s = ((int64_t)pmod(i0[0] - 1 + m1, n[0]) * n[1]
                     + pmod(i0[1] - 1 + m2, n[1])) * n[2]
                    + pmod(i0[2] - 1 + m3, n[2]);
        int64_t row = s * (int64_t)L;
        for (l = 0; l < L; ++l) {
            double are = coef_re(a, kind, row + l);
            if (!cplx) {
                if (val) val[l] += are * theta;
                if (grad) for (c = 0; c < 3; ++c) grad[c * L + l] += are * gth[c];
                if (lap) lap[l] += are * lth;
            } else {
                double aim = coef_im(a, kind, row + l);
                if (val) { val[2 * l] += are * theta; val[2 * l + 1] += aim * theta; }
                if (grad) for (c = 0; c < 3; ++c) {
                    grad[2 * (c * L + l)] += are * gth[c];
                    grad[2 * (c * L + l) + 1] += aim * gth[c];
                }
                if (lap) { lap[2 * l] += are * lth; lap[2 * l + 1] += aim * lth; }
            }
        }
    }

    /* Bloch factor for a k-point: psi = exp(i k.r) u with the unwrapped r. */
    if (cplx && kvec) {
        double kr = kvec[0] * r[0] + kvec[1] * r[1] + kvec[2] * r[2];
        double k2 = kvec[0] * kvec[0] + kvec[1] * kvec[1] + kvec[2] * kvec[2];
        double cr = cos(kr), ci = sin(kr);
        for (l = 0; l < L; ++l) {
            double ur = val ? val[2 * l] : 0.0, ui = val ? val[2 * l + 1] : 0.0;
            /* u (in val) is present whenever grad or lap is requested, and
             * grad u whenever lap is: oracle_eval checks both */
            double gr[3], gi[3];
            if (grad) for (c = 0; c < 3; ++c) {
                gr[c] = grad[2 * (c * L + l)];
                gi[c] = grad[2 * (c * L + l) + 1];
            }
            if (lap) {
                /* lap u + 2 i k.grad u - |k|^2 u */
                double kgr = 0.0, kgi = 0.0;
                for (c = 0; c < 3; ++c) { kgr += kvec[c] * gr[c]; kgi += kvec[c] * gi[c]; }
                double lr = lap[2 * l] - 2.0 * kgi - k2 * ur;
                double li = lap[2 * l + 1] + 2.0 * kgr - k2 * ui;
                lap[2 * l] = cr * lr - ci * li;
                lap[2 * l + 1] = cr * li + ci * lr;
            }
            if (grad) for (c = 0; c < 3; ++c) {
                /* grad u + i k u */
                double xr = gr[c] - kvec[c] * ui;
                double xi = gi[c] + kvec[c] * ur;
                grad[2 * (c * L + l)] = cr * xr - ci * xi;
                grad[2 * (c * L + l) + 1] = cr * xi + ci * xr;
            }
            if (val) {
                val[2 * l] = cr * ur - ci * ui;
                val[2 * l + 1] = cr * ui + ci * ur;
            }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Evaluate orbitals, gradients and Laplacians at npos positions.
 *   lattice  rows a_1, a_2, a_3 (bohr), row-major
 *   n1,n2,n3 grid points per lattice vector; norb orbitals L
 *   coef     [n1][n2][n3][L] C order, of the given kind (complex interleaved)
 *   kvec     NULL for the Gamma point / real orbitals
 *   pos      [npos][3] Cartesian bohr
 *   val      [npos][L], grad [npos][3][L], lap [npos][L] doubles (x2 when
 *            complex, interleaved); any of them may be NULL
 *   nthreads OpenMP threads over positions (<=0: all the runtime offers)
 * Returns 0, or -1 for bad arguments.  With a k-point the Bloch factor of
 * grad needs val, and that of lap needs val and grad; values only is fine. */
int oracle_eval(const double lattice[9], int n1, int n2, int n3, int norb,
                const void* coef, int kind, const double* kvec,
                const double* pos, int64_t npos,
                double* val, double* grad, double* lap, int nthreads)
{
    double G[9], M[9], g[9];
    int n[3] = {n1, n2, n3};
    int c, d, e;
    if (n1 < 1 || n2 < 1 || n3 < 1 || norb < 1 || npos < 0) return -1;
    if (kind < ORC_F64 || kind > ORC_C64) return -1;
    if (kvec && (kind == ORC_F64 || kind == ORC_F32)) return -1;
    /* with a Bloch factor, grad needs u and lap needs u and grad u */
    if (kvec && ((grad && !val) || (lap && (!val || !grad)))) return -1;
    if (oracle_inverse3(lattice, G) != 0) return -1;
    for (c = 0; c < 3; ++c)
        for (d = 0; d < 3; ++d) M[c * 3 + d] = (double)n[d] * G[c * 3 + d];
    for (d = 0; d < 3; ++d)
        for (e = 0; e < 3; ++e) {
            double s = 0.0;
            for (c = 0; c < 3; ++c) s += M[c * 3 + d] * M[c * 3 + e];
            g[d * 3 + e] = s;
        }
    const int w = (kind == ORC_C128 || kind == ORC_C64) ? 2 : 1;
    int64_t j;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) if (nthreads > 1)
    for (j = 0; j < npos; ++j) {
        eval_one(G, M, g, n, norb, coef, kind, kvec, pos + 3 * j,
                 val ? val + (size_t)w * norb * j : NULL,
                 grad ? grad + (size_t)w * 3 * norb * j : NULL,
                 lap ? lap + (size_t)w * norb * j : NULL);
    }
    return 0;
}
