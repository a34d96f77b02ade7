/*
 * Driver for the sanitizer build of the CPU oracle (test infrastructure).
 * Links oracle/oracle.c built with -fsanitize=address,undefined and calls
 * every exported function on small seeded inputs, including the edge cases
 * (length-1 chains, zero weights, one-node grids, a 3D grid), checking a few
 * invariants so that the run exercises every code path; the sanitizers report
 * any out-of-bounds access, leak or undefined behaviour and abort the run.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_tv1d(long m, const double *v, const double *a, double *x, double *p);
double orc_cut_energy(int ndim, const long *dims, const double *w, const double *const *a, const uint8_t *lab);
double orc_bruteforce(int ndim, const long *dims, const double *w, const double *const *a, uint8_t *min_set,
                      uint8_t *max_set, long *count);
double orc_mincut(int method, int ndim, const long *dims, const double *w, const double *const *a,
                  uint8_t *min_set, uint8_t *max_set, double *flow_out);
typedef struct {
    int32_t iters, status;
    double cert, energy, lower_bound, tv_gap, tau_used;
} orc_stats;
int orc_dr_solve(int ndim, const long *dims, const double *w, const double *const *a, int variant, int max_iters,
                 double gap_tol, double tv_tol, double tau0, const double *z0, double *x_out, uint8_t *labels_out,
                 double *z_out, double *cert_hist, double *tvgap_hist, orc_stats *st);
int orc_prox_family(int ndim, const long *dims, int axis, const double *v, const double *a_axis, double *x,
                    double *p);
int orc_lower_bound(int ndim, const long *dims, const double *w, const double *const *a, double *const *p,
                    double *lb, double *tvgap);

static uint64_t rng_state = 12345;
static double urand(void)  /* xorshift64*, uniform in [0, 1) */
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (double)((rng_state * 2685821657736338717ull) >> 11) / 9007199254740992.0;
}

static int fails = 0;
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++fails;                                                  \
        }                                                             \
    } while (0)

static void grid_case(int ndim, const long *dims, int with_bf)
{
    long n = 1;
    for (int j = 0; j < ndim; ++j) n *= dims[j];
    double *w = malloc(sizeof(double) * n);
    double *a[3] = {0, 0, 0};
    for (long i = 0; i < n; ++i) w[i] = floor(41 * urand()) - 20;
    for (int j = 0; j < ndim; ++j) {
        a[j] = malloc(sizeof(double) * n);
        for (long i = 0; i < n; ++i) a[j][i] = floor(11 * urand());
    }
    uint8_t *mn = malloc(n), *mx = malloc(n), *lab = malloc(n);
    double e_ek = orc_mincut(0, ndim, dims, w, (const double *const *)a, mn, mx, NULL);
    double e_di = orc_mincut(1, ndim, dims, w, (const double *const *)a, mn, mx, NULL);
    CHECK(e_ek == e_di);
    CHECK(orc_cut_energy(ndim, dims, w, (const double *const *)a, mn) == e_di);
    if (with_bf) {
        long cnt = 0;
        double e_bf = orc_bruteforce(ndim, dims, w, (const double *const *)a, mn, mx, &cnt);
        CHECK(e_bf == e_di && cnt >= 1);
    }
    double *x = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * 3 * n);
    double *ch = malloc(sizeof(double) * 400), *th = malloc(sizeof(double) * 400);
    orc_stats st;
    for (int variant = 0; variant < 2; ++variant) {
        if (variant == 0 && ndim != 2) continue;
        int rc = orc_dr_solve(ndim, dims, w, (const double *const *)a, variant, 400, 1e-3, 0.0, 1e-3, NULL, x, lab, z,
                              ch, th, &st);
        CHECK(rc == 0 && st.status == 0 && st.energy == e_di);
    }
    double *p[3];
    for (int j = 0; j < ndim; ++j) {
        p[j] = malloc(sizeof(double) * n);
        CHECK(orc_prox_family(ndim, dims, j, w, a[j], x, p[j]) == 0);
    }
    double lb = 0, gap = 0;
    CHECK(orc_lower_bound(ndim, dims, w, (const double *const *)a, p, &lb, &gap) == 0);
    CHECK(lb <= e_di + 1e-9 && gap >= -1e-9);
    for (int j = 0; j < ndim; ++j) { free(a[j]); free(p[j]); }
    free(w); free(mn); free(mx); free(lab); free(x); free(z); free(ch); free(th);
}

int main(void)
{
    /* chains: lengths 1..40, random, zero and huge weights */
    for (long m = 1; m <= 40; ++m) {
        for (int kind = 0; kind < 3; ++kind) {
            double *v = malloc(sizeof(double) * m), *a = malloc(sizeof(double) * (m > 1 ? m - 1 : 1));
            double *x = malloc(sizeof(double) * m), *p = malloc(sizeof(double) * (m > 1 ? m - 1 : 1));
            for (long i = 0; i < m; ++i) v[i] = 10 * urand() - 5;
            for (long i = 0; i + 1 < m; ++i) a[i] = kind == 0 ? 2 * urand() : (kind == 1 ? 0.0 : 1e6);
            CHECK(orc_tv1d(m, v, a, x, p) == 0);
            double sv = 0, sx = 0;
            for (long i = 0; i < m; ++i) { sv += v[i]; sx += x[i]; }
            CHECK(fabs(sv - sx) <= 1e-9 * (1 + fabs(sv)));
            free(v); free(a); free(x); free(p);
        }
    }
    long d1[2] = {1, 1}, d2[2] = {3, 4}, d3[2] = {12, 9}, d4[3] = {3, 4, 5}, d5[2] = {1, 7};
    grid_case(2, d1, 1);
    grid_case(2, d2, 1);
    grid_case(2, d5, 1);
    grid_case(2, d3, 0);
    grid_case(3, d4, 0);
    printf("oracle sanitizer driver: %d failed checks\n", fails);
    return fails != 0;
}
