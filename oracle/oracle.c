/*
 * FP64 CPU oracle for the RPM-FFT solver of Peng, Nepal & Dayal,
 * "Effective Response of Heterogeneous Materials using the Recursive
 * Projection Method", CMAME 364:112946 (2020).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the HIP path against a plain, slow
 * and obviously correct implementation.  It shares no code with the GPU
 * library.
 *
 * What it computes (each function cites the passage it follows):
 *   - complex DFTs: a naive O(n^2) DFT and a recursive decimation-in-time
 *     mixed-radix (2, 3, naive for other primes) FFT, applied axis by axis
 *     to full complex 3-D arrays (no half spectrum);
 *   - the isotropic reference-medium Green operator in Fourier space written
 *     as an explicit fourth-order tensor (the textbook Moulinec-Suquet form;
 *     the paper names the operator in Sec. 2, eqs. for the periodic Green
 *     function, without printing it);
 *   - the Lippmann-Schwinger fixed-point map F of Algorithm 1 / Sec. 3 (the
 *     equation of Sec. 3 that defines the fixed-point operator): FFT of BOTH the
 *     strain and the stress (the literal 18-transform form), the update
 *     eps_hat - Gamma:sigma_hat at k != 0, the mean strain E at k = 0, the
 *     inverse FFT, and the equilibrium error of Algorithm 1;
 *   - Algorithm 1 (basic fixed point) and Algorithm 2 (RPM-FFT) including the
 *     basis growth In(q, Z) of Sec. 3 (QR of two successive differences of q,
 *     one or two new columns);
 *   - the polarization (Accelerated FFT for alpha = beta = 2) iteration of
 *     Algorithm 3 / Sec. 5.5, with the sign of the reference-medium term of s_b
 *     taken as s_b = alpha sigma - beta C0:eps (as printed, s_b with +beta
 *     amplifies every fluctuation by -2 per step even for C = C0; the corrected
 *     scheme reaches the solution in one step there), and RPM around it
 *     (Algorithm 2 with F replaced by that iteration, Sec. 5.5).
 *
 * Conventions (readings of the paper, stated once):
 *   - fields are stored as [6][nz][ny][nx] real arrays, x fastest, tensor
 *     components in the order xx, yy, zz, yz, xz, xy (tensor, not
 *     engineering, shear);
 *   - forward DFT unnormalised with kernel exp(-2 pi i m.x/n); inverse
 *     carries 1/N;
 *   - wave vector in radians per voxel, k_j = 2 pi m_j / n_j with the signed
 *     index m_j in [-n_j/2, n_j/2); a Nyquist component takes -pi times the
 *     sign of the first non-Nyquist non-zero component in the order z, y, x
 *     (+1 if there is none) so that k(-m) = -k(m);
 *   - the equilibrium error is sqrt(sum_m |k.sigma_hat(m)|^2)/|sigma_hat(0)|
 *     (Frobenius norm; in-plane part of sigma_hat(0) when nz == 1), which is
 *     the real-space form sqrt(<|div sigma|^2>)/|<sigma>| of Algorithm 1;
 *   - inner products on fields are Frobenius sums over voxels
 *     (shear components weighted 2);
 *   - Newton on the unstable subspace uses H = Z^T F_u Z, bordered by one
 *     row and column per added basis vector, with F_u v = F(v; E = 0)
 *     (F is affine, so this is exact);
 *   - the basis grows after the fixed-point count nu exceeds n_max; one
 *     column is added when T22 <= kappa*T11, else two; every new column is
 *     projected onto zero-mean compatible fields (where differences of
 *     iterates lie in exact arithmetic), re-orthogonalised against Z twice
 *     (classical Gram-Schmidt, two passes) and dropped when its norm falls
 *     below 1e-10 of its norm before these projections.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORC_PI 3.14159265358979323846264338327950288

/* component index of the symmetric pair (i, j) in the 6-component layout */
static const int VOIGT_OF[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};

/* Frobenius weight of each stored component */
static const double FROB_W[6] = {1.0, 1.0, 1.0, 2.0, 2.0, 2.0};

static double delta(int i, int j) { return i == j ? 1.0 : 0.0; }

/* ------------------------------------------------------------------------ */
/* Discrete Fourier transforms                                              */
/* ------------------------------------------------------------------------ */

/* y[k] = sum_j x[j*stride] exp(sign 2 pi i j k / n), written out. */
void orc_dft_naive(const double *xin, double *yout, int n, int sign)
{
    const cplx *x = (const cplx *)xin;
    cplx *y = (cplx *)yout;
    for (int k = 0; k < n; ++k) {
        cplx s = 0.0;
        for (int j = 0; j < n; ++j) {
            long e = ((long)j * k) % n;
            double ang = sign * 2.0 * ORC_PI * (double)e / (double)n;
            s += x[j] * (cos(ang) + I * sin(ang));
        }
        y[k] = s;
    }
}

/* Recursive decimation-in-time FFT.  x is read with the given stride; the
 * length-len transform is written contiguously to y.  tw[e] holds
 * exp(sign 2 pi i e / n0) for the top-level length n0, and tws = n0/len
 * converts exponents of the current length to table indices. */
static void fft_rec(const cplx *x, long stride, cplx *y, int len, const cplx *tw, int tws, cplx *scratch)
{
    if (len == 1) {
        y[0] = x[0];
        return;
    }
    int p = (len % 2 == 0) ? 2 : (len % 3 == 0) ? 3 : 0;
    if (p == 0) {
        /* length with a prime factor other than 2 and 3: plain DFT sum */
        for (int k = 0; k < len; ++k) {
            cplx s = 0.0;
            for (int j = 0; j < len; ++j) s += x[j * stride] * tw[(((long)j * k) % len) * tws];
            scratch[k] = s;
        }
        memcpy(y, scratch, sizeof(cplx) * len);
        return;
    }
    int m = len / p;
    /* transforms of the p decimated subsequences x[r + p j] */
    for (int r = 0; r < p; ++r) fft_rec(x + r * stride, stride * p, y + r * m, m, tw, tws * p, scratch + len);
    /* butterflies: X[k + m s] = sum_r w^{r (k + m s)} Y_r[k] */
    for (int k = 0; k < m; ++k) {
        for (int s = 0; s < p; ++s) {
            int kk = k + m * s;
            cplx acc = 0.0;
            for (int r = 0; r < p; ++r) acc += y[r * m + k] * tw[(((long)r * kk) % len) * tws];
            scratch[kk] = acc;
        }
    }
    memcpy(y, scratch, sizeof(cplx) * len);
}

static cplx *make_twiddles(int n, int sign)
{
    cplx *tw = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    for (int e = 0; e < n; ++e) {
        double ang = sign * 2.0 * ORC_PI * (double)e / (double)n;
        tw[e] = cos(ang) + I * sin(ang);
    }
    return tw;
}

/* 1-D transform of a contiguous length-n complex array (interleaved re, im). */
void orc_fft1(const double *xin, double *yout, int n, int sign)
{
    cplx *tw = make_twiddles(n, sign);
    cplx *scratch = (cplx *)malloc(sizeof(cplx) * (size_t)(4 * n + 8));
    fft_rec((const cplx *)xin, 1, (cplx *)yout, n, tw, 1, scratch);
    free(scratch);
    free(tw);
}

/* In-place 3-D transform of one complex array [nz][ny][nx], axis by axis. */
static void fft3(cplx *a, int nx, int ny, int nz, int sign)
{
    int dims[3] = {nx, ny, nz};
    long strides[3] = {1, nx, (long)nx * ny};
    for (int ax = 0; ax < 3; ++ax) {
        int n = dims[ax];
        if (n == 1) continue;
        int o1 = (ax + 1) % 3, o2 = (ax + 2) % 3;
        long npencil = (long)dims[o1] * dims[o2];
        cplx *tw = make_twiddles(n, sign);
#pragma omp parallel
        {
            cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)n);
            cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)n);
            cplx *scratch = (cplx *)malloc(sizeof(cplx) * (size_t)(4 * n + 8));
#pragma omp for schedule(static)
            for (long pc = 0; pc < npencil; ++pc) {
                long i1 = pc % dims[o1], i2 = pc / dims[o1];
                long base = i1 * strides[o1] + i2 * strides[o2];
                for (int j = 0; j < n; ++j) buf[j] = a[base + j * strides[ax]];
                fft_rec(buf, 1, out, n, tw, 1, scratch);
                for (int j = 0; j < n; ++j) a[base + j * strides[ax]] = out[j];
            }
            free(scratch);
            free(out);
            free(buf);
        }
        free(tw);
    }
}

/* Exported wrapper: in-place 3-D complex transform (interleaved re, im). */
void orc_fft3(double *data, int nx, int ny, int nz, int sign) { fft3((cplx *)data, nx, ny, nz, sign); }

/* ------------------------------------------------------------------------ */
/* Wave vectors, stiffness and the Green operator                           */
/* ------------------------------------------------------------------------ */

static int signed_index(int m, int n) { return (m < (n + 1) / 2) ? m : m - n; }
static int is_nyquist(int m, int n) { return (n % 2 == 0) && (m == n / 2); }

/* Wave vector (radians per voxel) of DFT index (mx, my, mz); see header. */
void orc_wavevector(int nx, int ny, int nz, int mx, int my, int mz, double *k)
{
    int n[3] = {nx, ny, nz}, m[3] = {mx, my, mz};
    double sgn = 1.0;
    for (int ax = 2; ax >= 0; --ax) { /* order z, y, x */
        if (!is_nyquist(m[ax], n[ax]) && m[ax] != 0) {
            sgn = signed_index(m[ax], n[ax]) > 0 ? 1.0 : -1.0;
            break;
        }
    }
    for (int ax = 0; ax < 3; ++ax) {
        if (is_nyquist(m[ax], n[ax]))
            k[ax] = -ORC_PI * sgn;
        else
            k[ax] = 2.0 * ORC_PI * (double)signed_index(m[ax], n[ax]) / (double)n[ax];
    }
}

/* Isotropic stiffness C_ijkl = lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk). */
static double stiff(double lam, double mu, int i, int j, int k, int l)
{
    return lam * delta(i, j) * delta(k, l) + mu * (delta(i, k) * delta(j, l) + delta(i, l) * delta(j, k));
}

/* Green operator of the isotropic reference medium (lam0, mu0) at unit
 * direction nv = k/|k|:
 *   G_ijkl = (d_ki n_l n_j + d_li n_k n_j + d_kj n_l n_i + d_lj n_k n_i)/(4 mu0)
 *            - (lam0 + mu0)/(mu0 (lam0 + 2 mu0)) n_i n_j n_k n_l          */
static double green(const double *nv, double lam0, double mu0, int i, int j, int k, int l)
{
    double a = (delta(k, i) * nv[l] * nv[j] + delta(l, i) * nv[k] * nv[j] + delta(k, j) * nv[l] * nv[i] +
                delta(l, j) * nv[k] * nv[i]) /
               (4.0 * mu0);
    double b = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)) * nv[i] * nv[j] * nv[k] * nv[l];
    return a - b;
}

/* out_ij = sum_kl G_ijkl(k) s_kl for a complex symmetric tensor given as 6
 * components (interleaved re, im: 12 doubles); zero for k = 0. */
void orc_gamma_apply(const double *k, double lam0, double mu0, const double *s6, double *out6)
{
    const cplx *s = (const cplx *)s6;
    cplx *o = (cplx *)out6;
    double kk = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    for (int c = 0; c < 6; ++c) o[c] = 0.0;
    if (kk == 0.0) return;
    double nv[3] = {k[0] / kk, k[1] / kk, k[2] / kk};
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            cplx acc = 0.0;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) acc += green(nv, lam0, mu0, i, j, p, q) * s[VOIGT_OF[p][q]];
            o[VOIGT_OF[i][j]] = acc;
        }
}

/* sigma = C(x) : eps, voxel by voxel, written with the fourth-order tensor. */
void orc_stress(long N, const unsigned char *phase, const double *lame, const double *eps, double *sig)
{
    for (long x = 0; x < N; ++x) {
        double lam = lame[2 * phase[x]], mu = lame[2 * phase[x] + 1];
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j) {
                double acc = 0.0;
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q) acc += stiff(lam, mu, i, j, p, q) * eps[VOIGT_OF[p][q] * N + x];
                sig[VOIGT_OF[i][j] * N + x] = acc;
            }
    }
}

/* ------------------------------------------------------------------------ */
/* The Lippmann-Schwinger map F (the iteration body of Algorithm 1; Sec. 3)   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nx, ny, nz;
    long N;
    const unsigned char *phase;
    const double *lame; /* [n_phases][2] */
    double lam0, mu0;
    int map;             /* 0: Lippmann-Schwinger map F; 1: polarization iteration */
    double alpha, beta;  /* polarization parameters (Accelerated FFT: 2, 2) */
} problem;

static int gauss_solve(int n, const double *A_in, const double *b_in, double *y);
static void polarization_update(const problem *pr, const double *E6, const double *eps, const double *sig,
                                double *out);

/* xi = F(eps; E); *err = equilibrium error of eps; sig_avg = <C:eps>.
 * Returns the largest |imaginary part| left by the inverse transform. */
static double fmap(const problem *pr, const double *E6, const double *eps, double *xi, double *err, double *sig_avg)
{
    long N = pr->N;
    double *sig = (double *)malloc(sizeof(double) * 6 * (size_t)N);
    cplx *eh = (cplx *)malloc(sizeof(cplx) * 6 * (size_t)N);
    cplx *sh = (cplx *)malloc(sizeof(cplx) * 6 * (size_t)N);

    /* sigma = C(x):eps */
    orc_stress(N, pr->phase, pr->lame, eps, sig);
    /* eps_hat = FFT[eps], sigma_hat = FFT[sigma] */
    for (int c = 0; c < 6; ++c) {
        for (long x = 0; x < N; ++x) {
            eh[c * N + x] = eps[c * N + x];
            sh[c * N + x] = sig[c * N + x];
        }
        fft3(eh + c * N, pr->nx, pr->ny, pr->nz, -1);
        fft3(sh + c * N, pr->nx, pr->ny, pr->nz, -1);
    }

    /* error = sqrt(sum_m |k . sigma_hat|^2) / |sigma_hat(0)| */
    double num = 0.0;
    for (int mz = 0; mz < pr->nz; ++mz)
        for (int my = 0; my < pr->ny; ++my)
            for (int mx = 0; mx < pr->nx; ++mx) {
                long x = ((long)mz * pr->ny + my) * pr->nx + mx;
                double k[3];
                orc_wavevector(pr->nx, pr->ny, pr->nz, mx, my, mz, k);
                for (int i = 0; i < 3; ++i) {
                    cplx v = 0.0;
                    for (int j = 0; j < 3; ++j) v += k[j] * sh[VOIGT_OF[i][j] * N + x];
                    num += creal(v) * creal(v) + cimag(v) * cimag(v);
                }
            }
    double den = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            if (pr->nz == 1 && (i == 2 || j == 2)) continue; /* in-plane norm in 2-D */
            cplx v = sh[VOIGT_OF[i][j] * N];
            den += creal(v) * creal(v) + cimag(v) * cimag(v);
        }
    *err = sqrt(num) / sqrt(den);
    for (int c = 0; c < 6; ++c) sig_avg[c] = creal(sh[c * N]) / (double)N;

    /* xi_hat = eps_hat - Gamma(k):sigma_hat for k != 0 ; xi_hat(0) = N E */
    for (int mz = 0; mz < pr->nz; ++mz)
        for (int my = 0; my < pr->ny; ++my)
            for (int mx = 0; mx < pr->nx; ++mx) {
                long x = ((long)mz * pr->ny + my) * pr->nx + mx;
                if (x == 0) {
                    for (int c = 0; c < 6; ++c) eh[c * N] = (double)N * E6[c];
                    continue;
                }
                double k[3], s6[12], g6[12];
                orc_wavevector(pr->nx, pr->ny, pr->nz, mx, my, mz, k);
                for (int c = 0; c < 6; ++c) {
                    s6[2 * c] = creal(sh[c * N + x]);
                    s6[2 * c + 1] = cimag(sh[c * N + x]);
                }
                orc_gamma_apply(k, pr->lam0, pr->mu0, s6, g6);
                for (int c = 0; c < 6; ++c) eh[c * N + x] -= g6[2 * c] + I * g6[2 * c + 1];
            }

    double max_im = 0.0;
    if (pr->map == 1) {
        /* the polarization iteration replaces the update (Algorithm 3) */
        polarization_update(pr, E6, eps, sig, xi);
        free(sh);
        free(eh);
        free(sig);
        return 0.0;
    }
    /* xi = F^{-1}[xi_hat] (1/N), real part */
    for (int c = 0; c < 6; ++c) {
        fft3(eh + c * N, pr->nx, pr->ny, pr->nz, +1);
        for (long x = 0; x < N; ++x) {
            cplx v = eh[c * N + x] / (double)N;
            xi[c * N + x] = creal(v);
            if (fabs(cimag(v)) > max_im) max_im = fabs(cimag(v));
        }
    }
    free(sh);
    free(eh);
    free(sig);
    return max_im;
}

/* Mandel 6x6 matrix of an isotropic stiffness (shear rows and columns carry
 * sqrt(2)), from the fourth-order tensor. */
static const int PAIR_I[6] = {0, 1, 2, 1, 0, 0}, PAIR_J[6] = {0, 1, 2, 2, 2, 1};
static double mandel_f(int a) { return a < 3 ? 1.0 : sqrt(2.0); }
static void mandel_stiff(double lam, double mu, double *M)
{
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b)
            M[a * 6 + b] = mandel_f(a) * mandel_f(b) * stiff(lam, mu, PAIR_I[a], PAIR_J[a], PAIR_I[b], PAIR_J[b]);
}

/* Algorithm 3, one iteration given eps and sigma = C:eps:
 *   s_a = sigma + (1 - beta) C0:eps,   s_b = alpha sigma - beta C0:eps,
 *   eb_hat = -Gamma0(k) : F[s_b] (k != 0),  eb_hat(0) = N beta E,
 *   eps+ = (C(x) + C0)^{-1} : (s_a + C0 : F^{-1}[eb_hat]),
 * the inverse taken voxel by voxel on the Mandel matrix. */
static void polarization_update(const problem *pr, const double *E6, const double *eps, const double *sig,
                                double *out)
{
    long N = pr->N;
    double *c0e = (double *)malloc(sizeof(double) * 6 * (size_t)N);
    double *eb = (double *)malloc(sizeof(double) * 6 * (size_t)N);
    double *sa = (double *)malloc(sizeof(double) * 6 * (size_t)N);
    cplx *sbh = (cplx *)malloc(sizeof(cplx) * 6 * (size_t)N);
    unsigned char *zero_ph = (unsigned char *)calloc((size_t)N, 1);
    double ref[2] = {pr->lam0, pr->mu0};
    orc_stress(N, zero_ph, ref, eps, c0e); /* C0 : eps */
    for (int c = 0; c < 6; ++c) {
        for (long x = 0; x < N; ++x) {
            sa[c * N + x] = sig[c * N + x] + (1.0 - pr->beta) * c0e[c * N + x];
            sbh[c * N + x] = pr->alpha * sig[c * N + x] - pr->beta * c0e[c * N + x];
        }
        fft3(sbh + c * N, pr->nx, pr->ny, pr->nz, -1);
    }
    for (int mz = 0; mz < pr->nz; ++mz)
        for (int my = 0; my < pr->ny; ++my)
            for (int mx = 0; mx < pr->nx; ++mx) {
                long x = ((long)mz * pr->ny + my) * pr->nx + mx;
                if (x == 0) {
                    for (int c = 0; c < 6; ++c) sbh[c * N] = (double)N * pr->beta * E6[c];
                    continue;
                }
                double k[3], s6[12], g6[12];
                orc_wavevector(pr->nx, pr->ny, pr->nz, mx, my, mz, k);
                for (int c = 0; c < 6; ++c) {
                    s6[2 * c] = creal(sbh[c * N + x]);
                    s6[2 * c + 1] = cimag(sbh[c * N + x]);
                }
                orc_gamma_apply(k, pr->lam0, pr->mu0, s6, g6);
                for (int c = 0; c < 6; ++c) sbh[c * N + x] = -(g6[2 * c] + I * g6[2 * c + 1]);
            }
    for (int c = 0; c < 6; ++c) {
        fft3(sbh + c * N, pr->nx, pr->ny, pr->nz, +1);
        for (long x = 0; x < N; ++x) eb[c * N + x] = creal(sbh[c * N + x]) / (double)N;
    }
    orc_stress(N, zero_ph, ref, eb, c0e); /* C0 : eps_b (c0e reused) */
    double M0[36];
    mandel_stiff(pr->lam0, pr->mu0, M0);
    for (long x = 0; x < N; ++x) {
        double M[36], rhs[6], y[6];
        mandel_stiff(pr->lame[2 * pr->phase[x]], pr->lame[2 * pr->phase[x] + 1], M);
        for (int a = 0; a < 36; ++a) M[a] += M0[a];
        for (int a = 0; a < 6; ++a) rhs[a] = mandel_f(a) * (sa[a * N + x] + c0e[a * N + x]);
        gauss_solve(6, M, rhs, y);
        for (int a = 0; a < 6; ++a) out[a * N + x] = y[a] / mandel_f(a);
    }
    free(zero_ph);
    free(sbh);
    free(sa);
    free(eb);
    free(c0e);
}

static void init_problem(problem *pr, int nx, int ny, int nz, const unsigned char *phase, const double *lame,
                         double lam0, double mu0)
{
    pr->nx = nx;
    pr->ny = ny;
    pr->nz = nz;
    pr->N = (long)nx * ny * nz;
    pr->phase = phase;
    pr->lame = lame;
    pr->lam0 = lam0;
    pr->mu0 = mu0;
    pr->map = 0;
    pr->alpha = 2.0;
    pr->beta = 2.0;
}

/* v <- Gamma0 * (C0 : v) with the k = 0 term removed: the projection onto
 * zero-mean compatible strain fields (Gamma0 C0 is the identity on
 * sym(k (x) a) at every k != 0 and annihilates the rest).  Every difference of
 * iterates lies in that space in exact arithmetic; the projection removes the
 * rounding residue that dominates such differences near convergence. */
static void project_compatible(const problem *pr, double *v)
{
    long N = pr->N;
    cplx *vh = (cplx *)malloc(sizeof(cplx) * 6 * (size_t)N);
    double *s = (double *)malloc(sizeof(double) * 6 * (size_t)N);
    double *ref = (double *)malloc(sizeof(double) * 2);
    unsigned char *zero_ph = (unsigned char *)calloc((size_t)N, 1);
    ref[0] = pr->lam0;
    ref[1] = pr->mu0;
    orc_stress(N, zero_ph, ref, v, s); /* C0 : v */
    for (int c = 0; c < 6; ++c) {
        for (long x = 0; x < N; ++x) vh[c * N + x] = s[c * N + x];
        fft3(vh + c * N, pr->nx, pr->ny, pr->nz, -1);
    }
    for (int mz = 0; mz < pr->nz; ++mz)
        for (int my = 0; my < pr->ny; ++my)
            for (int mx = 0; mx < pr->nx; ++mx) {
                long x = ((long)mz * pr->ny + my) * pr->nx + mx;
                double k[3], s6[12], g6[12];
                orc_wavevector(pr->nx, pr->ny, pr->nz, mx, my, mz, k);
                for (int c = 0; c < 6; ++c) {
                    s6[2 * c] = creal(vh[c * N + x]);
                    s6[2 * c + 1] = cimag(vh[c * N + x]);
                }
                orc_gamma_apply(k, pr->lam0, pr->mu0, s6, g6); /* zero at k = 0 */
                for (int c = 0; c < 6; ++c) vh[c * N + x] = g6[2 * c] + I * g6[2 * c + 1];
            }
    for (int c = 0; c < 6; ++c) {
        fft3(vh + c * N, pr->nx, pr->ny, pr->nz, +1);
        for (long x = 0; x < N; ++x) v[c * N + x] = creal(vh[c * N + x]) / (double)N;
    }
    free(zero_ph);
    free(ref);
    free(s);
    free(vh);
}

/* Exported: the compatible projection of one field (in place). */
void orc_project_compatible(int nx, int ny, int nz, double lam0, double mu0, double *v)
{
    problem pr;
    init_problem(&pr, nx, ny, nz, NULL, NULL, lam0, mu0);
    project_compatible(&pr, v);
}

/* Exported: one application of F (map 0) or of the polarization iteration
 * (map 1, parameters alpha, beta).  Returns the max imaginary residue (map 0). */
double orc_fmap(int nx, int ny, int nz, const unsigned char *phase, const double *lame, double lam0, double mu0,
                const double *E6, const double *eps, double *xi, double *err, double *sig_avg, int map,
                double alpha, double beta)
{
    problem pr;
    init_problem(&pr, nx, ny, nz, phase, lame, lam0, mu0);
    pr.map = map;
    pr.alpha = alpha;
    pr.beta = beta;
    return fmap(&pr, E6, eps, xi, err, sig_avg);
}

/* Exported: eps + alpha (C(x) + C0)^{-1} C0 : (F(eps) - eps), the form the
 * polarization iteration takes on compatible strain fields of mean E (used to
 * pin the iteration against the Lippmann-Schwinger map). */
void orc_polarization_reduced(int nx, int ny, int nz, const unsigned char *phase, const double *lame, double lam0,
                              double mu0, const double *E6, const double *eps, double alpha, double *out)
{
    problem pr;
    init_problem(&pr, nx, ny, nz, phase, lame, lam0, mu0);
    long N = pr.N;
    double *xi = (double *)malloc(sizeof(double) * 6 * (size_t)N);
    double err, sav[6];
    fmap(&pr, E6, eps, xi, &err, sav);
    double M0[36];
    mandel_stiff(lam0, mu0, M0);
    for (long x = 0; x < N; ++x) {
        double M[36], rhs[6], y[6];
        mandel_stiff(lame[2 * phase[x]], lame[2 * phase[x] + 1], M);
        for (int a = 0; a < 36; ++a) M[a] += M0[a];
        for (int a = 0; a < 6; ++a) {
            rhs[a] = 0.0;
            for (int b = 0; b < 6; ++b) rhs[a] += M0[a * 6 + b] * mandel_f(b) * (xi[b * N + x] - eps[b * N + x]);
        }
        gauss_solve(6, M, rhs, y);
        for (int a = 0; a < 6; ++a) out[a * N + x] = eps[a * N + x] + alpha * y[a] / mandel_f(a);
    }
    free(xi);
}

/* ------------------------------------------------------------------------ */
/* Small dense helpers                                                      */
/* ------------------------------------------------------------------------ */

static double fdot(long N, const double *a, const double *b)
{
    double s = 0.0;
    for (int c = 0; c < 6; ++c)
        for (long x = 0; x < N; ++x) s += FROB_W[c] * a[c * N + x] * b[c * N + x];
    return s;
}

/* Solve A y = b (A is n x n, row major, copied) by Gaussian elimination with
 * partial pivoting.  Returns 0, or 1 if a pivot is below 1e-14 max|A|. */
static int gauss_solve(int n, const double *A_in, const double *b_in, double *y)
{
    if (n == 0) return 0;
    double *A = (double *)malloc(sizeof(double) * n * n);
    double *b = (double *)malloc(sizeof(double) * n);
    memcpy(A, A_in, sizeof(double) * n * n);
    memcpy(b, b_in, sizeof(double) * n);
    double amax = 0.0;
    for (int i = 0; i < n * n; ++i)
        if (fabs(A[i]) > amax) amax = fabs(A[i]);
    int status = 0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (!(fabs(A[piv * n + c]) > 1e-14 * amax)) {
            status = 1;
            break;
        }
        if (piv != c) {
            for (int j = 0; j < n; ++j) {
                double t = A[c * n + j];
                A[c * n + j] = A[piv * n + j];
                A[piv * n + j] = t;
            }
            double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
            b[r] -= f * b[c];
        }
    }
    if (status == 0) {
        for (int r = n - 1; r >= 0; --r) {
            double s = b[r];
            for (int j = r + 1; j < n; ++j) s -= A[r * n + j] * y[j];
            y[r] = s / A[r * n + r];
        }
    }
    free(b);
    free(A);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Algorithms 1 and 2                                                       */
/* ------------------------------------------------------------------------ */

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_DIVERGED = 2, ORC_SINGULAR = 3 };

/* Add column v (6N, overwritten) to the basis Z (p columns, stride 6N) after
 * two classical Gram-Schmidt passes; norm0 is v's norm before projection.
 * Returns 1 if the column was added. */
static int add_column(long N, double *Z, int p, double *v, double norm0)
{
    long L = 6 * N;
    for (int pass = 0; pass < 2; ++pass) {
        double *coef = (double *)malloc(sizeof(double) * (p > 0 ? p : 1));
        for (int j = 0; j < p; ++j) coef[j] = fdot(N, Z + j * L, v);
        for (int j = 0; j < p; ++j)
            for (long i = 0; i < L; ++i) v[i] -= coef[j] * Z[j * L + i];
        free(coef);
    }
    double nv = sqrt(fdot(N, v, v));
    if (!(nv > 1e-10 * norm0)) return 0;
    for (long i = 0; i < L; ++i) Z[p * L + i] = v[i] / nv;
    return 1;
}

/*
 * One solve for the mean strain E (Algorithm 1 when scheme == 0, Algorithm 2
 * when scheme == 1).
 *
 * Z, W: caller buffers of p_max columns of 6N doubles; H: p_max*p_max.  On
 * entry *p holds the number of valid columns to reuse (basis carried over
 * from an earlier load case: F_u does not depend on E), on exit the new
 * count.  eps_out receives the iterate whose error met tol (the input of the
 * last F call).  replay (nullable, length replay_len) forces the number of
 * columns added at each growth event (0, 1 or 2); decisions (nullable,
 * capacity dec_cap) records the numbers actually added.  hist (nullable,
 * capacity hist_cap) records the error after every main-loop F call.
 * On return counters = {main-loop F calls (the initial one included), JVP F
 * calls, growth events, basis size} and res_out = {final error, largest
 * imaginary residue left by any inverse transform}.
 * map 1 replaces F by the polarization iteration of Algorithm 3 with
 * parameters alpha, beta (Sec. 5.5: RPM-Accelerated FFT for alpha = beta = 2);
 * its iterates are not compatible, so new basis columns are not projected.
 * Returns 0 converged, 1 not converged in max_iter F calls, 2 diverged
 * (non-finite error or error above 1e6 times the initial one), 3 singular
 * I - H.
 */
int orc_solve(int nx, int ny, int nz, const unsigned char *phase, const double *lame, double lam0, double mu0,
              const double *E6, int scheme, double tol, int max_iter, int n_max, int p_max, double kappa,
              const int *replay, int replay_len, const double *eps_init, double *Z, double *W, double *H, int *p_io,
              double *eps_out, double *sig_avg, int *counters, double *res_out, double *hist, int hist_cap,
              int *decisions, int dec_cap, int map, double alpha, double beta)
{
    problem pr;
    init_problem(&pr, nx, ny, nz, phase, lame, lam0, mu0);
    pr.map = map;
    pr.alpha = alpha;
    pr.beta = beta;
    long N = pr.N, L = 6 * N;
    int p = (scheme == 1) ? *p_io : 0;
    if (scheme == 0) p_max = 0;

    double *eps = (double *)malloc(sizeof(double) * L);
    double *xi = (double *)malloc(sizeof(double) * L);
    double *q[3];
    for (int i = 0; i < 3; ++i) q[i] = (double *)malloc(sizeof(double) * L);
    double *d1 = (double *)malloc(sizeof(double) * L);
    double *d2 = (double *)malloc(sizeof(double) * L);
    double zero6[6] = {0, 0, 0, 0, 0, 0};
    double max_im = 0.0, im;

    /* initialisation: eps^0 = E (or a supplied start), xi^0 = F(eps^0) */
    if (eps_init) {
        memcpy(eps, eps_init, sizeof(double) * L);
    } else {
        for (int c = 0; c < 6; ++c)
            for (long x = 0; x < N; ++x) eps[c * N + x] = E6[c];
    }
    double err, err0;
    im = fmap(&pr, E6, eps, xi, &err, sig_avg);
    if (im > max_im) max_im = im;
    err0 = err;
    int iters = 1, jvps = 0, growth = 0, nq = 0, nu = 0, status = ORC_NOT_CONVERGED, ndec = 0;
    if (hist && hist_cap > 0) hist[0] = err;

    double *zc = (double *)malloc(sizeof(double) * (p_max + 2));
    double *ze = (double *)malloc(sizeof(double) * (p_max + 2));
    double *rhs = (double *)malloc(sizeof(double) * (p_max + 2));
    double *y = (double *)malloc(sizeof(double) * (p_max + 2));
    double *IH = (double *)malloc(sizeof(double) * (p_max + 2) * (p_max + 2));

    for (;;) {
        if (!isfinite(err) || err > 1e6 * err0) {
            status = ORC_DIVERGED;
            break;
        }
        if (err <= tol) {
            status = ORC_OK;
            break;
        }
        if (iters >= max_iter) {
            status = ORC_NOT_CONVERGED;
            break;
        }

        /* project to the unstable subspace: z = Z^T eps, zeta = Z^T xi */
        for (int j = 0; j < p; ++j) {
            ze[j] = fdot(N, Z + j * L, eps);
            zc[j] = fdot(N, Z + j * L, xi);
        }
        /* Newton step z' = z + (I - H)^{-1} (zeta - z) */
        for (int i = 0; i < p; ++i) {
            rhs[i] = zc[i] - ze[i];
            for (int j = 0; j < p; ++j) IH[i * p + j] = delta(i, j) - H[i * p_max + j];
        }
        if (gauss_solve(p, IH, rhs, y)) {
            status = ORC_SINGULAR;
            break;
        }
        /* q = xi - Z zeta ; eps = Z z' + q */
        double *qn = q[nq % 3];
        memcpy(qn, xi, sizeof(double) * L);
        for (int j = 0; j < p; ++j)
            for (long i = 0; i < L; ++i) qn[i] -= zc[j] * Z[j * L + i];
        memcpy(eps, qn, sizeof(double) * L);
        for (int j = 0; j < p; ++j) {
            double zn = ze[j] + y[j];
            for (long i = 0; i < L; ++i) eps[i] += zn * Z[j * L + i];
        }
        ++nq;
        /* fixed-point iteration on the whole space */
        im = fmap(&pr, E6, eps, xi, &err, sig_avg);
        if (im > max_im) max_im = im;
        if (hist && iters < hist_cap) hist[iters] = err;
        ++iters;
        ++nu;

        /* basis growth once nu exceeds n_max (skipped once converged: it
         * cannot change the returned iterate) */
        if (nu > n_max && p < p_max && err > tol && isfinite(err) && err <= 1e6 * err0 && iters < max_iter) {
            int want = 0;
            int ncol = 0;
            if (nq >= 2) {
                /* D = [dq^(nu), dq^(nu-1)] from the last three q's */
                double *qa = q[(nq - 1) % 3], *qb = q[(nq - 2) % 3];
                for (long i = 0; i < L; ++i) d1[i] = qa[i] - qb[i];
                double T11 = sqrt(fdot(N, d1, d1)), T22 = 0.0;
                int have2 = 0;
                if (nq >= 3) {
                    double *qc = q[(nq - 3) % 3];
                    for (long i = 0; i < L; ++i) d2[i] = qb[i] - qc[i];
                    have2 = 1;
                }
                if (T11 > 0.0) {
                    /* modified Gram-Schmidt QR of D */
                    for (long i = 0; i < L; ++i) d1[i] /= T11;
                    if (have2) {
                        double T12 = fdot(N, d1, d2);
                        for (long i = 0; i < L; ++i) d2[i] -= T12 * d1[i];
                        T22 = sqrt(fdot(N, d2, d2));
                    }
                    want = (have2 && T22 > kappa * T11) ? 2 : 1;
                }
                if (replay && growth < replay_len) want = replay[growth];
                /* the classical map keeps every iterate compatible with mean E, so
                 * its differences are zero-mean compatible fields and the projection
                 * only removes rounding residue; the polarization iterates are not
                 * compatible, and their differences are kept as they are */
                if (want >= 1 && T11 > 0.0) {
                    if (pr.map == 0) project_compatible(&pr, d1);
                    if (add_column(N, Z, p, d1, 1.0)) {
                        ++p;
                        ++ncol;
                    }
                }
                if (want >= 2 && have2 && T22 > 0.0 && p < p_max) {
                    for (long i = 0; i < L; ++i) d2[i] /= T22;
                    if (pr.map == 0) project_compatible(&pr, d2);
                    if (add_column(N, Z, p, d2, 1.0)) {
                        ++p;
                        ++ncol;
                    }
                }
            }
            /* H: one new column of F_u Z per added vector (JVP = F(v; 0)) */
            for (int c = p - ncol; c < p; ++c) {
                double e_dummy, s_dummy[6];
                im = fmap(&pr, zero6, Z + c * L, W + c * L, &e_dummy, s_dummy);
                if (im > max_im) max_im = im;
                ++jvps;
                for (int i = 0; i <= c; ++i) H[i * p_max + c] = fdot(N, Z + i * L, W + c * L);
                for (int j = 0; j < c; ++j) H[c * p_max + j] = fdot(N, Z + c * L, W + j * L);
            }
            if (decisions && ndec < dec_cap) decisions[ndec] = ncol;
            ++ndec;
            ++growth;
            nu = 0;
            nq = 0;
        }
    }

    memcpy(eps_out, eps, sizeof(double) * L);
    if (scheme == 1) *p_io = p;
    counters[0] = iters;
    counters[1] = jvps;
    counters[2] = growth;
    counters[3] = p;
    res_out[0] = err;
    res_out[1] = max_im;

    free(IH);
    free(y);
    free(rhs);
    free(ze);
    free(zc);
    free(d2);
    free(d1);
    for (int i = 0; i < 3; ++i) free(q[i]);
    free(xi);
    free(eps);
    return status;
}

/*
 * Seed the unstable-subspace basis with given vectors (a warm start of Z; any
 * orthonormal Z with H = Z^T F_u Z serves the Newton step of Sec. 3).  Each of
 * the p0 vectors V[k] (6N doubles, read only) goes through the steps basis
 * growth applies to a difference of iterates: normalised, projected onto
 * zero-mean compatible fields (map 0), added after two classical Gram-Schmidt
 * passes (dropped below 1e-10 of its norm), then its JVP column of W
 * (F(z; E = 0)) and its border of H.  Z, W, H and *p_io as in orc_solve: the
 * *p_io columns already held are kept and new ones appended up to p_max.
 * Returns the number of columns added.
 */
int orc_seed_basis(int nx, int ny, int nz, const unsigned char *phase, const double *lame, double lam0, double mu0,
                   const double *V, int p0, int p_max, double *Z, double *W, double *H, int *p_io, int map,
                   double alpha, double beta)
{
    problem pr;
    init_problem(&pr, nx, ny, nz, phase, lame, lam0, mu0);
    pr.map = map;
    pr.alpha = alpha;
    pr.beta = beta;
    long N = pr.N, L = 6 * N;
    int p = *p_io, added = 0;
    double *v = (double *)malloc(sizeof(double) * L);
    double zero6[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < p0 && p < p_max; ++k) {
        memcpy(v, V + k * L, sizeof(double) * L);
        double nv = sqrt(fdot(N, v, v));
        if (!(nv > 0.0)) continue;
        for (long i = 0; i < L; ++i) v[i] /= nv;
        if (map == 0) project_compatible(&pr, v);
        if (!add_column(N, Z, p, v, 1.0)) continue;
        double e_dummy, s_dummy[6];
        fmap(&pr, zero6, Z + p * L, W + p * L, &e_dummy, s_dummy);
        for (int i = 0; i <= p; ++i) H[i * p_max + p] = fdot(N, Z + i * L, W + p * L);
        for (int j = 0; j < p; ++j) H[p * p_max + j] = fdot(N, Z + p * L, W + j * L);
        ++p;
        ++added;
    }
    *p_io = p;
    free(v);
    return added;
}
