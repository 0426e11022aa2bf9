/*
 * Driver for the host sanitizer build of the CPU oracle (test infrastructure):
 * compiled together with oracle/oracle.c under -fsanitize=address,undefined and
 * run by tests/test_sanitizers.py.  It walks every exported routine on small
 * grids (odd and even extents, 2-D and 3-D, the polarization map, basis growth
 * with both decisions, a carried and a seeded basis) so that an out-of-bounds
 * access or undefined behaviour anywhere in them stops the run.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_dft_naive(const double *xin, double *yout, int n, int sign);
void orc_fft1(const double *xin, double *yout, int n, int sign);
void orc_fft3(double *data, int nx, int ny, int nz, int sign);
void orc_wavevector(int nx, int ny, int nz, int mx, int my, int mz, double *k);
void orc_gamma_apply(const double *k, double lam0, double mu0, const double *s6, double *out6);
void orc_stress(long N, const unsigned char *phase, const double *lame, const double *eps, double *sig);
void orc_project_compatible(int nx, int ny, int nz, double lam0, double mu0, double *v);
double orc_fmap(int nx, int ny, int nz, const unsigned char *phase, const double *lame, double lam0, double mu0,
                const double *E6, const double *eps, double *xi, double *err, double *sig_avg, int map, double alpha,
                double beta);
void orc_polarization_reduced(int nx, int ny, int nz, const unsigned char *phase, const double *lame, double lam0,
                              double mu0, const double *E6, const double *eps, double alpha, double *out);
int orc_solve(int nx, int ny, int nz, const unsigned char *phase, const double *lame, double lam0, double mu0,
              const double *E6, int scheme, double tol, int max_iter, int n_max, int p_max, double kappa,
              const int *replay, int replay_len, const double *eps_init, double *Z, double *W, double *H, int *p_io,
              double *eps_out, double *sig_avg, int *counters, double *res_out, double *hist, int hist_cap,
              int *decisions, int dec_cap, int map, double alpha, double beta);
int orc_seed_basis(int nx, int ny, int nz, const unsigned char *phase, const double *lame, double lam0, double mu0,
                   const double *V, int p0, int p_max, double *Z, double *W, double *H, int *p_io, int map,
                   double alpha, double beta);

static unsigned long long rng = 88172645463325252ull;
static double urand(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static int run_grid(int nx, int ny, int nz, int map)
{
    const long N = (long)nx * ny * nz, L = 6 * N;
    unsigned char *ph = malloc((size_t)N);
    for (long i = 0; i < N; ++i) ph[i] = (unsigned char)(urand() * 2.999);
    const double lame[6] = {0.58, 0.38, 4.0, 2.8, 0.1, 0.07};
    const double E[6] = {0.01, -0.002, nz > 1 ? 0.003 : 0.0, 0.0, 0.0, 0.002};
    double *eps = malloc(sizeof(double) * L), *xi = malloc(sizeof(double) * L), *sig = malloc(sizeof(double) * L);
    for (long i = 0; i < L; ++i) eps[i] = 0.01 * (urand() - 0.5);
    double err, sav[6];
    orc_fmap(nx, ny, nz, ph, lame, 2.0, 1.4, E, eps, xi, &err, sav, map, 2.0, 2.0);
    orc_stress(N, ph, lame, eps, sig);
    orc_project_compatible(nx, ny, nz, 2.0, 1.4, eps);
    if (map == 0) orc_polarization_reduced(nx, ny, nz, ph, lame, 2.0, 1.4, E, eps, 2.0, xi);
    const int pmax = 6;
    double *Z = calloc((size_t)pmax * L, sizeof(double)), *W = calloc((size_t)pmax * L, sizeof(double));
    double *H = calloc((size_t)pmax * pmax, sizeof(double)), hist[64];
    int p = 0, cnt[4], dec[16];
    double res[2];
    int st = orc_solve(nx, ny, nz, ph, lame, 2.0, 1.4, E, 1, 1e-12, 40, 3, pmax, 0.1, NULL, 0, NULL, Z, W, H, &p, eps,
                       sav, cnt, res, hist, 64, dec, 16, map, 2.0, 2.0);
    /* carried basis, forced decisions, supplied start */
    const int replay[3] = {2, 1, 0};
    st |= orc_solve(nx, ny, nz, ph, lame, 2.0, 1.4, E, 1, 1e-12, 30, 2, pmax, 0.1, replay, 3, eps, Z, W, H, &p, xi,
                    sav, cnt, res, hist, 64, dec, 16, map, 2.0, 2.0);
    p = 0;
    orc_seed_basis(nx, ny, nz, ph, lame, 2.0, 1.4, eps, 1, pmax, Z, W, H, &p, map, 2.0, 2.0);
    free(H);
    free(W);
    free(Z);
    free(sig);
    free(xi);
    free(eps);
    free(ph);
    return st < 0;
}

int main(void)
{
    for (int n = 1; n <= 12; ++n) {
        double x[24], y[24], z[24];
        for (int i = 0; i < 2 * n; ++i) x[i] = urand();
        orc_dft_naive(x, y, n, -1);
        orc_fft1(x, z, n, -1);
        orc_fft1(z, y, n, +1);
    }
    double a[2 * 4 * 6 * 3];
    for (int i = 0; i < 2 * 4 * 6 * 3; ++i) a[i] = urand();
    orc_fft3(a, 4, 6, 3, -1);
    double k[3], s6[12], o6[12];
    for (int i = 0; i < 12; ++i) s6[i] = urand();
    orc_wavevector(8, 6, 5, 4, 3, 2, k);
    orc_gamma_apply(k, 2.0, 1.4, s6, o6);
    const int grids[][3] = {{4, 6, 1}, {5, 3, 1}, {4, 4, 4}, {3, 5, 6}, {6, 4, 2}};
    int bad = 0;
    for (unsigned g = 0; g < sizeof grids / sizeof grids[0]; ++g)
        for (int map = 0; map < 2; ++map) bad |= run_grid(grids[g][0], grids[g][1], grids[g][2], map);
    printf("oracle driver done\n");
    return bad;
}
