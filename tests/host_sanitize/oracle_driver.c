/* oracle_driver.c -- runs every entry point of the CPU oracle (oracle/fv_oracle.c)
 * on small seeded batches, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer: 2D and 3D, every supported unknown count, patch
 * sizes from 1 to the largest the tests use, periodic or not, patches at
 * shuffled offsets with gaps, halos from neighbours, per-patch step sizes and
 * the generic solver for every built-in PDE.  Results are checked by the pin
 * tests; here the sanitizers check the oracle's memory accesses and arithmetic.
 * Exit status 0 when every call returned 0. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int fvo_batch_update(const double *in, double *out, const int32_t *sizes, const int64_t *offsets,
                     int32_t num_patches, int32_t dim, int32_t nq, double dt, double h, double gamma,
                     int32_t periodic, double *lambda_out, int32_t nthreads);
int fvo_batch_lambda(const double *state, const int32_t *sizes, const int64_t *offsets, int32_t num_patches,
                     int32_t dim, int32_t nq, double gamma, double *lambda_out);
int fvo_batch_wrap(double *state, const int32_t *sizes, const int64_t *offsets, int32_t num_patches, int32_t dim,
                   int32_t nq);
int fvo_halo_fill(const double *src, double *dst, const int32_t *sizes, const int64_t *offsets,
                  const int32_t *neighbors, int32_t num_patches, int32_t dim, int32_t nq);
int fvo_batch_update_lts(const double *in, double *out, const int32_t *sizes, const int64_t *offsets,
                         int32_t num_patches, int32_t dim, int32_t nq, const double *dt, const double *h,
                         double gamma, double *lambda_out, int32_t nthreads);
int fvo_local_dt(const double *lambda, const double *h, int32_t num_patches, int32_t dim, double cfl,
                 double *dt_out);
void fvo_flux(const double *q, int32_t n, int32_t nq, double gamma, double *f, double *lam);
void fvo_rusanov(const double *qL, const double *qR, int32_t n, int32_t nq, double gamma, double *fhat);
int fvo_pde_shape(int32_t pde, int32_t dim, int32_t *nq, int32_t *nv, int32_t *nprm);
int fvo_pde_update(int32_t pde, const double *prm, int32_t nprm, const double *in, double *out,
                   const int32_t *sizes, const int64_t *offsets, int32_t num_patches, int32_t dim, double dt, double h,
                   int32_t periodic, double *lambda_out);
int fvo_pde_terms(int32_t pde, int32_t dim, const double *prm, const double *q, int32_t n, const double *dq,
                  double *f, double *lam, double *b, double *s);

static int failures = 0;
#define CHECK(call)                                                        \
    do {                                                                   \
        if ((call) != 0) {                                                 \
            fprintf(stderr, "line %d: %s returned non-zero\n", __LINE__, #call); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand(void) { /* xorshift64*: a deterministic stream of [0, 1) */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (double)((rng_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static int64_t pdoubles(int p, int dim, int nq) {
    int64_t w = p + 2;
    return (dim == 2 ? w * w : w * w * w) * nq;
}

/* A physical state in every volume: rho > 0, pressure > 0 (Euler); positive depth (shallow water). */
static void fill(double *a, int64_t nvol, int nq, int euler) {
    for (int64_t v = 0; v < nvol; ++v) {
        double *q = a + v * nq;
        for (int c = 0; c < nq; ++c) q[c] = urand() - 0.5;
        q[0] = 1.0 + 0.5 * urand();
        if (euler) q[nq - 1] = 3.0 + urand();
    }
}

/* T patches with sizes from `choices`, placed in reverse order with gaps. */
static int64_t layout(int T, const int *choices, int nch, int dim, int nq, int32_t *sizes, int64_t *offs) {
    int64_t pos = 0;
    for (int t = 0; t < T; ++t) sizes[t] = choices[(t * 7 + 3) % nch];
    for (int t = T - 1; t >= 0; --t) {
        pos += t % 3;
        offs[t] = pos;
        pos += pdoubles(sizes[t], dim, nq);
    }
    return pos + 2;
}

static void euler_cases(void) {
    const int c2[] = {1, 2, 3, 5, 9, 16, 17, 31, 64}, c3[] = {1, 2, 4, 5, 8, 13};
    for (int dim = 2; dim <= 3; ++dim) {
        for (int nq = 4; nq <= 5; ++nq) {
            if (dim == 3 && nq == 4) continue;
            const int *ch = dim == 2 ? c2 : c3;
            const int nch = dim == 2 ? 9 : 6, T = dim == 2 ? 40 : 14;
            int32_t sizes[64];
            int64_t offs[64];
            const int64_t n = layout(T, ch, nch, dim, nq, sizes, offs);
            double *a = malloc(sizeof(double) * n), *b = malloc(sizeof(double) * n);
            double lam[64], dt[64], h[64];
            fill(a, n / nq, nq, 1);
            memcpy(b, a, sizeof(double) * n);
            for (int periodic = 0; periodic <= 1; ++periodic) {
                CHECK(fvo_batch_update(a, b, sizes, offs, T, dim, nq, 1e-3, 1.0 / 48, 1.4, periodic, lam, 1));
                CHECK(fvo_batch_update(a, b, sizes, offs, T, dim, nq, 1e-3, 1.0 / 48, 1.4, periodic, NULL, 3));
            }
            CHECK(fvo_batch_lambda(a, sizes, offs, T, dim, nq, 1.4, lam));
            CHECK(fvo_batch_wrap(b, sizes, offs, T, dim, nq));
            for (int t = 0; t < T; ++t) {
                h[t] = 1.0 / (48 + t);
                dt[t] = 1e-4 * (1 + t % 3);
            }
            CHECK(fvo_batch_update_lts(a, b, sizes, offs, T, dim, nq, dt, h, 1.4, lam, 2));
            CHECK(fvo_local_dt(lam, h, T, dim, 0.4, dt));
            double q[5] = {1.1, 0.2, -0.1, 0.05, 2.5}, q2[5] = {0.9, -0.1, 0.3, 0.0, 2.2}, f[5], l, fh[5];
            for (int ax = 0; ax < dim; ++ax) {
                fvo_flux(q, ax, nq, 1.4, f, &l);
                fvo_rusanov(q, q2, ax, nq, 1.4, fh);
            }
            free(a);
            free(b);
        }
    }
    /* halos from neighbours: a 4 x 4 (2D) / 3 x 3 x 3 (3D) periodic tiling of one size */
    for (int dim = 2; dim <= 3; ++dim) {
        const int n = dim == 2 ? 4 : 3, p = dim == 2 ? 5 : 4, T = dim == 2 ? n * n : n * n * n;
        int32_t sizes[27], nb[27 * 6];
        int64_t offs[27];
        for (int t = 0; t < T; ++t) {
            sizes[t] = p;
            offs[t] = t * pdoubles(p, dim, 5);
            int c[3] = {t % n, (t / n) % n, t / (n * n)};
            for (int a = 0; a < dim; ++a)
                for (int s = 0; s < 2; ++s) {
                    int d[3] = {c[0], c[1], c[2]};
                    d[a] = (d[a] + (s ? 1 : n - 1)) % n;
                    nb[t * 2 * dim + 2 * a + s] = d[0] + n * (d[1] + n * d[2]);
                }
        }
        nb[0] = -1; /* one face without a neighbour */
        const int64_t N = T * pdoubles(p, dim, 5);
        double *a = malloc(sizeof(double) * N), *b = malloc(sizeof(double) * N);
        fill(a, N / 5, 5, 1);
        memcpy(b, a, sizeof(double) * N);
        CHECK(fvo_halo_fill(a, b, sizes, offs, nb, T, dim, 5));
        free(a);
        free(b);
    }
}

static void pde_cases(void) {
    const double prm[5][4] = {{1.4, 0, 0, 0}, {9.81, 0.5, 0, 0}, {0.7, -0.4, 0.25, 0}, {1.2, 2.0, 0, 0},
                              {1.2, 2.0, 0, 0}};
    for (int pde = 0; pde <= 4; ++pde) {
        for (int dim = 2; dim <= 3; ++dim) {
            int32_t nq, nv, np;
            if (fvo_pde_shape(pde, dim, &nq, &nv, &np) != 0) continue; /* shallow water is 2D only */
            const int ch[] = {1, 3, 6, 11};
            const int T = 9;
            int32_t sizes[9];
            int64_t offs[9];
            const int64_t n = layout(T, ch, 4, dim, nq, sizes, offs);
            double *a = malloc(sizeof(double) * n), *b = malloc(sizeof(double) * n), lam[9];
            fill(a, n / nq, nq, pde == 0);
            memcpy(b, a, sizeof(double) * n);
            for (int periodic = 0; periodic <= 1; ++periodic)
                CHECK(fvo_pde_update(pde, prm[pde], np, a, b, sizes, offs, T, dim, 1e-4, 1.0 / 48, periodic, lam));
            double q[5], dq[5], f[5], l, bb[5], s[5];
            for (int c = 0; c < nq; ++c) {
                q[c] = 1.0 + 0.1 * c;
                dq[c] = 0.01 * (c + 1);
            }
            if (pde == 0) q[nq - 1] = 3.0;
            for (int ax = 0; ax < dim; ++ax) CHECK(fvo_pde_terms(pde, dim, prm[pde], q, ax, dq, f, &l, bb, s));
            free(a);
            free(b);
        }
    }
}

int main(void) {
    euler_cases();
    pde_cases();
    if (failures) {
        fprintf(stderr, "%d oracle calls failed\n", failures);
        return 1;
    }
    printf("ok: oracle entry points under the sanitizers\n");
    return 0;
}
