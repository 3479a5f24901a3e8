/* Drives every entry point of the oracle (oracle/lbo.c) on small lattices of
 * each configuration the tests use, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Exits 0 when every
 * call returns; the sanitizers abort on the first invalid access. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct lbo_lattice lbo_lattice;
lbo_lattice *lbo_create(const double *dp, const int *ip);
void lbo_destroy(lbo_lattice *L);
int lbo_set_regions(lbo_lattice *L, const int *blo, const int *bhi);
int lbo_update_regions(lbo_lattice *L, const int *blo, const int *bhi);
void lbo_init_equilibrium_t(lbo_lattice *L, const double *rho, const double *ux, const double *uy, const double *T);
void lbo_step(lbo_lattice *L, long nsteps);
void lbo_moments(const lbo_lattice *L, double *rho, double *ux, double *uy);
void lbo_conservation(const lbo_lattice *L, double *out);
void lbo_thermal(const lbo_lattice *L, double *T, double *qx, double *qy);
double lbo_energy(const lbo_lattice *L);
void lbo_indicator(const lbo_lattice *L, double *B);
void lbo_bands_from_indicator(const lbo_lattice *L, const double *B, double theta, int bmin, int bmax, int *blo,
                              int *bhi);
void lbo_set_closure(lbo_lattice *L, const double *c);
void lbo_get_populations(const lbo_lattice *L, int s, double *f);
void lbo_set_populations(lbo_lattice *L, int s, const double *f);
void lbo_project(int ns, int ords, int nd, int ordd, const double *fs, const double *closure, double *fd);
void lbo_project_t(int ns, int ords, int nd, int ordd, const double *fs, const double *closure, double *fd);
void lbo_equilibrium_t(int n, int order, double rho, double ux, double uy, double T, double *feq);
void lbo_force_t(int n, int order, double rho, double ux, double uy, double T, double gx, double gy, double *g);
void lbo_moments_node_t(int n, const double *f, double *rho, double *ux, double *uy, double *T);
void lbo_heat_flux_node(int n, const double *f, double *qx, double *qy);
void lbo_hermite_coeffs(int n, const double *f, double *a);
void lbo_from_coeffs(int n, const double *a, double *f);
double lbo_face_value(double nu, double fm1, double f0, double fp1, double fp2);
void lbo_set_threads(int n);

/* one case: nx, ny, n_low, eq_low, n_high, eq_high, tau_mode, xbc, ybc, iface,
 * tile_w, thermal, band_lo, band_hi, rho_in, rho_out, shear */
typedef struct {
    int nx, ny, nl, el, nh, eh, tau, xbc, ybc, iface, tw, th, lo, hi;
    double rin, rout, shear;
} kase;

static int run(const kase *c)
{
    double dp[16] = {0.1, 1.0, 0.09, 1e-5, -1e-5, -0.03, 0.0, 0.03, 0.0, c->rin, c->rout, 0.0, 0.0, c->shear,
                     1.05, 0.97};
    int ip[14] = {c->nx, c->ny, c->nl, c->nh, c->el, c->eh, c->el, c->eh, c->tau, c->xbc, c->ybc, c->iface, c->tw,
                  c->th};
    lbo_lattice *L = lbo_create(dp, ip);
    if (!L) return 1;
    int nt = (c->nx + c->tw - 1) / c->tw;
    int *lo = calloc(nt, sizeof(int)), *hi = calloc(nt, sizeof(int));
    for (int t = 0; t < nt; ++t) {
        lo[t] = c->iface ? c->lo : c->lo + t % 3;
        hi[t] = c->iface ? c->hi : c->hi + (t + 1) % 2;
    }
    lbo_set_regions(L, lo, hi);
    size_t N = (size_t)(c->ny + 1) * c->nx;
    double *r = malloc(N * sizeof(double)), *u = malloc(N * sizeof(double)), *v = malloc(N * sizeof(double));
    double *T = malloc(N * sizeof(double)), *B = malloc(N * sizeof(double));
    for (size_t k = 0; k < N; ++k) {
        double x = (double)(k % c->nx), y = (double)(k / c->nx);
        r[k] = 1.0 + 0.02 * sin(0.3 * x + 0.2 * y);
        u[k] = 0.02 * cos(0.2 * y);
        v[k] = 0.01 * sin(0.1 * x);
        T[k] = 1.0 + 0.03 * cos(0.25 * x - 0.1 * y);
    }
    lbo_init_equilibrium_t(L, r, u, v, T);
    lbo_step(L, 3);
    double out[3];
    lbo_moments(L, r, u, v);
    lbo_conservation(L, out);
    lbo_thermal(L, T, u, v);
    double e = lbo_energy(L);
    lbo_indicator(L, B);
    lbo_bands_from_indicator(L, B, 1e-3, 1, c->ny / 3, lo, hi);
    if (!c->iface) {
        size_t nq = (size_t)c->nh * c->nh * N;
        double *cl = malloc(nq * sizeof(double));
        for (size_t k = 0; k < nq; ++k) cl[k] = 1e-4 * (double)(k % 7);
        lbo_set_closure(L, cl);
        free(cl);
        lbo_update_regions(L, lo, hi);
        lbo_set_closure(L, NULL);
        lbo_step(L, 2);
    }
    double *f = malloc((size_t)c->nh * c->nh * N * sizeof(double));
    lbo_get_populations(L, 1, f);
    lbo_set_populations(L, 1, f);
    lbo_step(L, 1);
    free(f);
    int bad = !isfinite(out[0]) || !isfinite(e);
    free(r); free(u); free(v); free(T); free(B); free(lo); free(hi);
    lbo_destroy(L);
    return bad;
}

int main(void)
{
    lbo_set_threads(2);
    const kase cases[] = {
        {70, 24, 3, 2, 6, 4, 0, 0, 0, 0, 64, 0, 4, 5, 1.0, 1.0, 0.0},    /* coupled, walls, Hermite */
        {70, 24, 3, 2, 4, 3, 1, 1, 0, 0, 32, 0, 3, 3, 1.2, 1.0, 0.0},    /* pressure, tau ~ 1/rho, tiles */
        {40, 30, 3, 2, 6, 4, 0, 0, 0, 1, 40, 0, 5, 6, 1.0, 1.0, 0.0},    /* paper interface */
        {30, 20, 4, 3, 6, 4, 0, 0, 1, 0, 30, 0, 3, 4, 1.0, 1.0, 0.0},    /* periodic y */
        {24, 30, 3, 2, 6, 4, 0, 0, 2, 0, 24, 0, 6, 0, 1.0, 1.0, 1e-3},   /* imposed shear */
        {50, 24, 3, 2, 6, 4, 1, 0, 0, 0, 50, 1, 4, 4, 1.0, 1.0, 0.0},    /* thermal, Hermite */
        {40, 30, 3, 2, 4, 3, 0, 0, 0, 1, 40, 1, 5, 5, 1.0, 1.0, 0.0},    /* thermal, paper interface */
        {60, 20, 4, 3, 6, 4, 1, 1, 0, 0, 30, 1, 3, 3, 1.1, 1.0, 0.0},    /* thermal pressure channel */
    };
    int fails = 0;
    for (size_t k = 0; k < sizeof(cases) / sizeof(cases[0]); ++k) fails += run(&cases[k]);
    double fs[36], fd[36], a[36], rho, ux, uy, T, qx, qy;
    lbo_equilibrium_t(6, 4, 1.1, 0.1, -0.05, 1.2, fs);
    lbo_project(6, 4, 3, 2, fs, NULL, fd);
    lbo_project_t(3, 2, 6, 4, fd, NULL, fs);
    lbo_force_t(4, 3, 1.0, 0.1, 0.0, 1.1, 1e-3, 0.0, fd);
    lbo_moments_node_t(6, fs, &rho, &ux, &uy, &T);
    lbo_heat_flux_node(6, fs, &qx, &qy);
    lbo_hermite_coeffs(6, fs, a);
    lbo_from_coeffs(6, a, fd);
    (void)lbo_face_value(0.4, 1.0, 2.0, 2.5, 2.7);
    (void)lbo_face_value(-0.4, 1.0, 2.0, 2.0, 2.7);
    printf("cases %zu failures %d\n", sizeof(cases) / sizeof(cases[0]), fails);
    return fails != 0;
}
