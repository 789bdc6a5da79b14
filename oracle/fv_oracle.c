/*
 * fv_oracle.c -- plain FP64 CPU oracle for one explicit Euler step of the
 * Rusanov Finite Volume scheme over a batch of halo-padded Cartesian patches
 * (compressible Euler equations).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * It is written as the plain definition of the scheme, with no blocking,
 * fusion or reordering:
 *   - the update of a volume c over one time step (paper, Sec. 2.2, the
 *     unnumbered update formula):
 *         Q_new(c) = Q(c) + (dt/h) * sum_n [ Fhat_n(c - e_n/2) - Fhat_n(c + e_n/2) ]
 *     i.e. the flux through the left face enters with "+", the flux through
 *     the right face with "-" (Alg. 1, the two update microkernels);
 *   - the Rusanov face flux (Eq. 2):
 *         Fhat = 1/2 (F_n(Q_L) + F_n(Q_R)) - 1/2 max(lambda_n(Q_L), lambda_n(Q_R)) (Q_R - Q_L)
 *   - the user terms F_n (flux along axis n) and lambda_max,n (largest wave
 *     speed along n) of the compressible Euler equations, the PDE the paper's
 *     experiments solve (Sec. 5, N = 2 + d; Eq. 1 with B = S = delta = 0);
 *   - the per-patch maximum eigenvalue of the NEW solution that feeds the CFL
 *     condition (end of Sec. 2.2).
 *
 * Readings of the paper where it is garbled or silent (all listed in the
 * design notes of the repository):
 *   - Eq. 2 prints the dissipation as (C/h)(Q+ - Q-) max(lambda); the
 *     textbook Rusanov / local Lax-Friedrichs flux has C = 1/2 and no 1/h, and
 *     that is what is computed here.
 *   - The update formula prints "Delta t * h"; a conservative update of a
 *     volume of size h^d through faces of size h^(d-1) scales by dt/h.
 *   - lambda_max,n is the largest eigenvalue MAGNITUDE |u_n| + c.
 *   - the face wave speeds use the OLD state; the final reduction uses the
 *     new one.
 *   - only face halo volumes are ever read: corner (2D) and edge/corner (3D)
 *     halo volumes do not enter the result.
 *   - the difference of the two face fluxes is formed first, then the
 *     directional differences are summed in axis order ((x + y) + z), then
 *     scaled by dt/h and added to Q.
 *   - unknowns: N = 5 (rho, m_x, m_y, m_z, E) in 2D and 3D -- in 2D m_z is a
 *     passive momentum (advected, no z flux, part of the kinetic energy) --
 *     or the paper's N = 2 + d = 4 in 2D (rho, m_x, m_y, E).
 *   - max() propagates NaN (any NaN in, NaN out).
 *
 * Layout: patch t starts at offsets[t] (in doubles).  Its (p+2)^d volumes are
 * stored in x-fastest order, each volume holding its N unknowns contiguously
 * (array of structures):  index = offsets[t] + ((k*(p+2) + j)*(p+2) + i)*N + q,
 * with i, j, k in [0, p+1]; halo volumes sit at 0 and p+1.
 *
 * Compile with -O2 -ffp-contract=off and no fast-math: every operation below
 * rounds once, in the order written.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_MAXQ 5

/* NaN-propagating maximum: if either argument is NaN the result is NaN. */
static double ora_max(double a, double b)
{
    if (a != a) return a;
    if (b != b) return b;
    return (a > b) ? a : b;
}

/* Number of momentum components stored in a volume with nq unknowns. */
static int ora_nmom(int nq) { return nq - 2; }

/* Pressure of the ideal gas: p = (gamma - 1) (E - |m|^2 / (2 rho)). */
static double ora_pressure(const double *q, int nq, double gamma)
{
    double rho = q[0];
    double m2 = 0.0;
    for (int a = 0; a < ora_nmom(nq); ++a) m2 = m2 + q[1 + a] * q[1 + a];
    double E = q[nq - 1];
    return (gamma - 1.0) * (E - 0.5 * m2 / rho);
}

/*
 * User term F_n(Q) of the Euler equations along axis n, and
 * lambda_max,n(Q) = |u_n| + c with c = sqrt(gamma p / rho).
 *   F_n = ( m_n,  m_a u_n + p delta_{a n} (each stored momentum a),  (E + p) u_n )
 */
static void ora_flux(const double *q, int n, int nq, double gamma,
                     double *f, double *lam)
{
    double rho = q[0];
    double p = ora_pressure(q, nq, gamma);
    double un = q[1 + n] / rho;
    f[0] = q[1 + n];
    for (int a = 0; a < ora_nmom(nq); ++a) {
        double v = q[1 + a] * un;
        if (a == n) v = v + p;
        f[1 + a] = v;
    }
    f[nq - 1] = (q[nq - 1] + p) * un;
    double c = sqrt(gamma * p / rho);
    *lam = fabs(un) + c;
}

/* Rusanov flux through the face between left volume qL and right volume qR
 * along axis n (Eq. 2, with the reading C = 1/2 and no 1/h). */
static void ora_rusanov(const double *qL, const double *qR, int n, int nq,
                        double gamma, double *fhat)
{
    double fL[ORA_MAXQ], fR[ORA_MAXQ], lL, lR;
    ora_flux(qL, n, nq, gamma, fL, &lL);
    ora_flux(qR, n, nq, gamma, fR, &lR);
    double s = ora_max(lL, lR);
    for (int q = 0; q < nq; ++q)
        fhat[q] = 0.5 * (fL[q] + fR[q]) - 0.5 * s * (qR[q] - qL[q]);
}

/* Offset (in doubles) of volume (i, j, k) inside a padded patch. */
static size_t ora_vol(int p, int dim, int i, int j, int k, int nq)
{
    size_t w = (size_t)(p + 2);
    size_t kk = (dim == 3) ? (size_t)k : 0;
    return ((kk * w + (size_t)j) * w + (size_t)i) * (size_t)nq;
}

/* Largest wave speed over the interior volumes of one padded patch state:
 * max over interior c and axes n < dim of lambda_max,n(Q(c)). */
static double ora_patch_lambda(const double *P, int p, int dim, int nq, double gamma)
{
    double lmax = 0.0;
    int kend = (dim == 3) ? p : 1;
    int kbeg = (dim == 3) ? 1 : 0;
    for (int k = kbeg; k <= kend; ++k)
        for (int j = 1; j <= p; ++j)
            for (int i = 1; i <= p; ++i) {
                const double *q = P + ora_vol(p, dim, i, j, k, nq);
                for (int n = 0; n < dim; ++n) {
                    double f[ORA_MAXQ], lam;
                    ora_flux(q, n, nq, gamma, f, &lam);
                    lmax = ora_max(lmax, lam);
                }
            }
    return lmax;
}

/* Periodic self-wrap of the face halo of one output patch: on each axis the
 * halo layer at 0 takes the interior layer at p and the halo layer at p+1 the
 * interior layer at 1.  Faces only: corner / edge halo volumes are untouched. */
static void ora_wrap_faces(double *P, int p, int dim, int nq)
{
    int kbeg = (dim == 3) ? 1 : 0, kend = (dim == 3) ? p : 0;
    for (int k = kbeg; k <= kend; ++k)
        for (int j = 1; j <= p; ++j) {
            memcpy(P + ora_vol(p, dim, 0, j, k, nq), P + ora_vol(p, dim, p, j, k, nq), sizeof(double) * nq);
            memcpy(P + ora_vol(p, dim, p + 1, j, k, nq), P + ora_vol(p, dim, 1, j, k, nq), sizeof(double) * nq);
        }
    for (int k = kbeg; k <= kend; ++k)
        for (int i = 1; i <= p; ++i) {
            memcpy(P + ora_vol(p, dim, i, 0, k, nq), P + ora_vol(p, dim, i, p, k, nq), sizeof(double) * nq);
            memcpy(P + ora_vol(p, dim, i, p + 1, k, nq), P + ora_vol(p, dim, i, 1, k, nq), sizeof(double) * nq);
        }
    if (dim == 3)
        for (int j = 1; j <= p; ++j)
            for (int i = 1; i <= p; ++i) {
                memcpy(P + ora_vol(p, dim, i, j, 0, nq), P + ora_vol(p, dim, i, j, p, nq), sizeof(double) * nq);
                memcpy(P + ora_vol(p, dim, i, j, p + 1, nq), P + ora_vol(p, dim, i, j, 1, nq), sizeof(double) * nq);
            }
}

/* One explicit Euler step of one patch: Q_new over the interior. */
static void ora_patch_step(const double *Pin, double *Pout, int p, int dim, int nq,
                           double dt, double h, double gamma)
{
    double r = dt / h;
    int kbeg = (dim == 3) ? 1 : 0, kend = (dim == 3) ? p : 0;
    for (int k = kbeg; k <= kend; ++k)
        for (int j = 1; j <= p; ++j)
            for (int i = 1; i <= p; ++i) {
                const int c[3] = {i, j, k};
                double D[ORA_MAXQ];
                for (int n = 0; n < dim; ++n) {
                    int lo[3] = {c[0], c[1], c[2]}, hi[3] = {c[0], c[1], c[2]};
                    lo[n] -= 1;
                    hi[n] += 1;
                    const double *qc = Pin + ora_vol(p, dim, c[0], c[1], c[2], nq);
                    const double *ql = Pin + ora_vol(p, dim, lo[0], lo[1], lo[2], nq);
                    const double *qh = Pin + ora_vol(p, dim, hi[0], hi[1], hi[2], nq);
                    double fleft[ORA_MAXQ], fright[ORA_MAXQ];
                    ora_rusanov(ql, qc, n, nq, gamma, fleft);   /* face c - e_n/2 */
                    ora_rusanov(qc, qh, n, nq, gamma, fright);  /* face c + e_n/2 */
                    for (int q = 0; q < nq; ++q) {
                        double d = fleft[q] - fright[q];
                        D[q] = (n == 0) ? d : D[q] + d;
                    }
                }
                const double *qc = Pin + ora_vol(p, dim, i, j, k, nq);
                double *qo = Pout + ora_vol(p, dim, i, j, k, nq);
                for (int q = 0; q < nq; ++q) qo[q] = qc[q] + r * D[q];
            }
}

/*
 * Batch entry point.  in/out: flat arrays holding every padded patch at
 * offsets[t]; out gets the new interior of every patch (and, when periodic is
 * non-zero, its self-wrapped face halo); lambda_out (may be NULL) gets the
 * maximum wave speed of the new interior of every patch.  nthreads <= 0 uses
 * the OpenMP default.  Returns 0, or -1 for arguments the oracle does not
 * cover.
 */
int fvo_batch_update(const double *in, double *out, const int32_t *sizes,
                     const int64_t *offsets, int32_t num_patches, int32_t dim,
                     int32_t nq, double dt, double h, double gamma, int32_t periodic,
                     double *lambda_out, int32_t nthreads)
{
    if (!(dim == 2 || dim == 3)) return -1;
    if (!(nq == 5 || (dim == 2 && nq == 4))) return -1;
    if (num_patches < 0) return -1;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
    for (int32_t t = 0; t < num_patches; ++t) {
        int p = sizes[t];
        const double *Pin = in + offsets[t];
        double *Pout = out + offsets[t];
        ora_patch_step(Pin, Pout, p, dim, nq, dt, h, gamma);
        if (periodic) ora_wrap_faces(Pout, p, dim, nq);
        if (lambda_out) lambda_out[t] = ora_patch_lambda(Pout, p, dim, nq, gamma);
    }
    (void)nthreads;
    return 0;
}

/* Maximum wave speed of the interior of every patch of a state (used for the
 * first time step size, before any update has produced a new solution). */
int fvo_batch_lambda(const double *state, const int32_t *sizes, const int64_t *offsets,
                     int32_t num_patches, int32_t dim, int32_t nq, double gamma,
                     double *lambda_out)
{
    if (!(dim == 2 || dim == 3)) return -1;
    if (!(nq == 5 || (dim == 2 && nq == 4))) return -1;
    for (int32_t t = 0; t < num_patches; ++t)
        lambda_out[t] = ora_patch_lambda(state + offsets[t], sizes[t], dim, nq, gamma);
    return 0;
}

/* Periodic self-wrap of the face halos of every patch of a state, in place. */
int fvo_batch_wrap(double *state, const int32_t *sizes, const int64_t *offsets,
                   int32_t num_patches, int32_t dim, int32_t nq)
{
    if (!(dim == 2 || dim == 3)) return -1;
    for (int32_t t = 0; t < num_patches; ++t)
        ora_wrap_faces(state + offsets[t], sizes[t], dim, nq);
    return 0;
}

/*
 * Face-halo fill from the neighbouring patches of a conforming patch mesh:
 * the step before the update that equips each patch with its halo layer
 * (Sec. 2.2).  neighbors[t*2d + 2n + s] is the patch that touches patch t
 * across its face on axis n, side s (s = 0: the face at coordinate 0, s = 1:
 * the face at p+1), or -1 for a face without a neighbour, whose halo volumes
 * are left as they are.  The halo layer on side 0 of axis n takes the
 * neighbour's interior layer at p (the layer next to their common face), the
 * halo layer on side 1 the neighbour's interior layer at 1; the coordinates
 * along the other axes are the same in both patches.  Faces only: corner /
 * edge halo volumes are untouched.  Values are read from src and written to
 * dst (which may be src itself: only interior volumes are read, only halo
 * volumes written).  Returns -1 when a neighbour has another size.
 */
int fvo_halo_fill(const double *src, double *dst, const int32_t *sizes, const int64_t *offsets,
                  const int32_t *neighbors, int32_t num_patches, int32_t dim, int32_t nq)
{
    if (!(dim == 2 || dim == 3)) return -1;
    for (int32_t t = 0; t < num_patches; ++t) {
        int p = sizes[t];
        for (int n = 0; n < dim; ++n)
            for (int s = 0; s < 2; ++s) {
                int32_t nb = neighbors[(size_t)t * 2 * dim + 2 * n + s];
                if (nb < 0) continue;
                if (sizes[nb] != p) return -1;
                /* every volume (i, j, k) of the face: coordinate n fixed, the others 1..p */
                int kbeg = (dim == 3) ? 1 : 0, kend = (dim == 3) ? p : 0;
                for (int k = kbeg; k <= kend; ++k)
                    for (int j = 1; j <= p; ++j)
                        for (int i = 1; i <= p; ++i) {
                            int h[3] = {i, j, k}, g[3] = {i, j, k};
                            if (n == 0 && i != 1) continue;  /* axis n takes one value per face */
                            if (n == 1 && j != 1) continue;
                            if (n == 2 && k != 1) continue;
                            h[n] = (s == 0) ? 0 : p + 1;    /* halo volume of patch t */
                            g[n] = (s == 0) ? p : 1;        /* interior volume of the neighbour */
                            memcpy(dst + offsets[t] + ora_vol(p, dim, h[0], h[1], h[2], nq),
                                   src + offsets[nb] + ora_vol(p, dim, g[0], g[1], g[2], nq), sizeof(double) * nq);
                        }
            }
    }
    return 0;
}

/*
 * One explicit Euler step of every patch with its own step size and mesh
 * width: patch t advances by dt[t] with volumes of width h[t] (local time
 * stepping: each patch has its own CFL-limited step, end of Sec. 2.2).  The
 * face halos are taken as they are in `in` (filled beforehand, e.g. by
 * fvo_halo_fill); out gets the new interiors, lambda_out (may be NULL) the
 * maximum wave speed of each new interior.
 */
int fvo_batch_update_lts(const double *in, double *out, const int32_t *sizes, const int64_t *offsets,
                         int32_t num_patches, int32_t dim, int32_t nq, const double *dt, const double *h,
                         double gamma, double *lambda_out, int32_t nthreads)
{
    if (!(dim == 2 || dim == 3)) return -1;
    if (!(nq == 5 || (dim == 2 && nq == 4))) return -1;
    if (num_patches < 0) return -1;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
    for (int32_t t = 0; t < num_patches; ++t) {
        int p = sizes[t];
        ora_patch_step(in + offsets[t], out + offsets[t], p, dim, nq, dt[t], h[t], gamma);
        if (lambda_out) lambda_out[t] = ora_patch_lambda(out + offsets[t], p, dim, nq, gamma);
    }
    (void)nthreads;
    return 0;
}

/*
 * Per-patch CFL step size from the patch's maximum wave speed (local time
 * stepping):  dt[t] = cfl * h[t] / (d * lambda[t]).  The same expression
 * as the global step size, per patch.
 */
int fvo_local_dt(const double *lambda, const double *h, int32_t num_patches, int32_t dim, double cfl,
                 double *dt_out)
{
    if (!(dim == 2 || dim == 3)) return -1;
    for (int32_t t = 0; t < num_patches; ++t) dt_out[t] = cfl * h[t] / (dim * lambda[t]);
    return 0;
}

/* Single-volume user terms, exposed so tests can evaluate F_n and lambda_n of
 * a given state directly. */
void fvo_flux(const double *q, int32_t n, int32_t nq, double gamma, double *f, double *lam)
{
    ora_flux(q, n, nq, gamma, f, lam);
}

/* Single-face Rusanov flux, exposed for tests. */
void fvo_rusanov(const double *qL, const double *qR, int32_t n, int32_t nq, double gamma,
                 double *fhat)
{
    ora_rusanov(qL, qR, n, nq, gamma, fhat);
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int32_t fvo_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ========================================================================
 * The generic solver of Eq. 1: the same step assembled from a PDE's user
 * terms -- flux F_n, non-conservative product B_n(Q) dQ/dx_n, source S and
 * largest wave speed lambda_max,n (Sec. 2.2: the user provides these and the
 * engine assembles the solver).  Point sources (the delta terms) are not
 * covered.
 *
 * Readings (the paper omits the treatment of B in the flux, Sec. 2.2):
 *   - the conservative part is Eq. 2 over the evolved unknowns;
 *   - B enters at every face as the jump B_n(Qbar) (Q_R - Q_L) with the face
 *     average Qbar = (Q_L + Q_R) / 2, half of it charged to each of the two
 *     volumes (the central, path-conservative discretisation of
 *     -B dQ/dx), so the volume right of the face receives
 *         G+ = Fhat - 1/2 B_n(Qbar) (Q_R - Q_L)
 *     and the volume left of it loses
 *         G- = Fhat + 1/2 B_n(Qbar) (Q_R - Q_L);
 *     with B = 0 both are Fhat and the step is the Euler step above;
 *   - the update of a volume is, difference first and in axis order,
 *         Q_new = Q + (dt/h) sum_n [G+_n(c - e_n/2) - G-_n(c + e_n/2)] + dt S(Q)
 *     (explicit Euler for the source, evaluated on the old state);
 *   - a PDE may carry parameters as unknowns (the bathymetry of the shallow
 *     water equations): the unknowns from nv on are not evolved, they keep
 *     their values and enter only through F, B, S and lambda.
 *
 * The PDEs (parameters in prm[]):
 *   FVO_PDE_EULER          the Euler equations of the first part, N = 5;
 *                          prm = {gamma}.
 *   FVO_PDE_SHALLOW_WATER  2D shallow water over a bathymetry b, Q = (h, hu,
 *                          hv, b), nv = 3; prm = {g, f}:
 *                            F_x = (hu, hu u, hv u),  F_y = (hv, hu v, hv v)
 *                            B_x dQ/dx = (0, g h d(h + b)/dx, 0)
 *                            B_y dQ/dy = (0, 0, g h d(h + b)/dy)
 *                            S = (0, f hv, -f hu)          (Coriolis)
 *                            lambda_n = |u_n| + sqrt(g h)
 *                          (the hydrostatic pressure is written as a
 *                          non-conservative product, so a lake at rest has no
 *                          momentum change).
 *   FVO_PDE_ADVECTION      dq/dt + a . grad q = 0, N = 1; prm = {a_x, a_y, a_z};
 *                          F_n = a_n q, lambda_n = |a_n|.
 *   FVO_PDE_ACOUSTICS      linear acoustics, Q = (p, u_1 .. u_d), N = 1 + d;
 *                          prm = {rho0, K0}:  F_n = (K0 u_n, p / rho0 e_n),
 *                          lambda_n = sqrt(K0 / rho0).
 *   FVO_PDE_ACOUSTICS_NCP  the same system written as B_n dQ/dx_n with F = 0.
 * ====================================================================== */

#define FVO_PDE_EULER 0
#define FVO_PDE_SHALLOW_WATER 1
#define FVO_PDE_ADVECTION 2
#define FVO_PDE_ACOUSTICS 3
#define FVO_PDE_ACOUSTICS_NCP 4

typedef struct {
    int nq, nv;  /* unknowns per volume; the first nv are evolved */
    /* F_n(Q) over the evolved unknowns; NULL: no flux */
    void (*flux)(const double *q, int n, const double *prm, double *f);
    double (*eig)(const double *q, int n, const double *prm);
    /* B_n(qbar) dq over the evolved unknowns; NULL: no non-conservative term */
    void (*ncp)(const double *qbar, const double *dq, int n, const double *prm, double *b);
    /* S(Q) over the evolved unknowns; NULL: no source */
    void (*source)(const double *q, const double *prm, double *s);
} ora_pde;

static void pde_euler_flux(const double *q, int n, const double *prm, double *f)
{
    double lam;
    ora_flux(q, n, 5, prm[0], f, &lam);
}

static double pde_euler_eig(const double *q, int n, const double *prm)
{
    double f[ORA_MAXQ], lam;
    ora_flux(q, n, 5, prm[0], f, &lam);
    return lam;
}

static void pde_swe_flux(const double *q, int n, const double *prm, double *f)
{
    double un = q[n + 1] / q[0];
    f[0] = q[n + 1];
    f[1] = q[1] * un;
    f[2] = q[2] * un;
    (void)prm;
}

static double pde_swe_eig(const double *q, int n, const double *prm)
{
    return fabs(q[1 + n] / q[0]) + sqrt(prm[0] * q[0]);
}

static void pde_swe_ncp(const double *qbar, const double *dq, int n, const double *prm, double *b)
{
    double hydro = prm[0] * qbar[0] * (dq[0] + dq[3]);  /* g h d(h + b) */
    b[0] = 0.0;
    b[1] = (n == 0) ? hydro : 0.0;
    b[2] = (n == 1) ? hydro : 0.0;
}

static void pde_swe_source(const double *q, const double *prm, double *s)
{
    s[0] = 0.0;
    s[1] = prm[1] * q[2];
    s[2] = -prm[1] * q[1];
}

static void pde_adv_flux(const double *q, int n, const double *prm, double *f) { f[0] = prm[n] * q[0]; }

static double pde_adv_eig(const double *q, int n, const double *prm)
{
    (void)q;
    return fabs(prm[n]);
}

static int ora_acoustic_dim;  /* set per call: the number of velocity components */

static void pde_ac_flux(const double *q, int n, const double *prm, double *f)
{
    f[0] = prm[1] * q[1 + n];
    for (int a = 0; a < ora_acoustic_dim; ++a) f[1 + a] = (a == n) ? q[0] / prm[0] : 0.0;
}

static double pde_ac_eig(const double *q, int n, const double *prm)
{
    (void)q;
    (void)n;
    return sqrt(prm[1] / prm[0]);
}

static void pde_ac_ncp(const double *qbar, const double *dq, int n, const double *prm, double *b)
{
    (void)qbar;
    b[0] = prm[1] * dq[1 + n];
    for (int a = 0; a < ora_acoustic_dim; ++a) b[1 + a] = (a == n) ? dq[0] / prm[0] : 0.0;
}

/* The PDE `pde` in `dim` dimensions and the number of parameters it takes;
 * -1 if there is no such PDE. */
static int ora_pde_get(int pde, int dim, ora_pde *P, int *nprm)
{
    if (!(dim == 2 || dim == 3)) return -1;
    memset(P, 0, sizeof(*P));
    switch (pde) {
    case FVO_PDE_EULER:
        P->nq = P->nv = 5;
        P->flux = pde_euler_flux;
        P->eig = pde_euler_eig;
        *nprm = 1;
        return 0;
    case FVO_PDE_SHALLOW_WATER:
        if (dim != 2) return -1;
        P->nq = 4;
        P->nv = 3;
        P->flux = pde_swe_flux;
        P->eig = pde_swe_eig;
        P->ncp = pde_swe_ncp;
        P->source = pde_swe_source;
        *nprm = 2;
        return 0;
    case FVO_PDE_ADVECTION:
        P->nq = P->nv = 1;
        P->flux = pde_adv_flux;
        P->eig = pde_adv_eig;
        *nprm = 3;
        return 0;
    case FVO_PDE_ACOUSTICS:
    case FVO_PDE_ACOUSTICS_NCP:
        ora_acoustic_dim = dim;
        P->nq = P->nv = 1 + dim;
        if (pde == FVO_PDE_ACOUSTICS) P->flux = pde_ac_flux;
        else P->ncp = pde_ac_ncp;
        P->eig = pde_ac_eig;
        *nprm = 2;
        return 0;
    default:
        return -1;
    }
}

/* The two face values of Eq. 2 with the non-conservative jump: gplus for the
 * volume right of the face, gminus for the one left of it. */
static void ora_pde_face(const ora_pde *P, const double *qL, const double *qR, int n, const double *prm,
                         double *gplus, double *gminus)
{
    double fL[ORA_MAXQ], fR[ORA_MAXQ];
    for (int q = 0; q < P->nv; ++q) fL[q] = fR[q] = 0.0;
    if (P->flux) {
        P->flux(qL, n, prm, fL);
        P->flux(qR, n, prm, fR);
    }
    double s = ora_max(P->eig(qL, n, prm), P->eig(qR, n, prm));
    double b[ORA_MAXQ];
    if (P->ncp) {
        double qbar[ORA_MAXQ], dq[ORA_MAXQ];
        for (int q = 0; q < P->nq; ++q) {
            qbar[q] = 0.5 * (qL[q] + qR[q]);
            dq[q] = qR[q] - qL[q];
        }
        P->ncp(qbar, dq, n, prm, b);
    }
    for (int q = 0; q < P->nv; ++q) {
        double fhat = 0.5 * (fL[q] + fR[q]) - 0.5 * s * (qR[q] - qL[q]);
        gplus[q] = P->ncp ? fhat - 0.5 * b[q] : fhat;
        gminus[q] = P->ncp ? fhat + 0.5 * b[q] : fhat;
    }
}

static void ora_pde_patch_step(const ora_pde *P, const double *Pin, double *Pout, int p, int dim,
                               double dt, double h, const double *prm)
{
    int nq = P->nq;
    const double ratio = dt / h;
    int kbeg = (dim == 3) ? 1 : 0, kend = (dim == 3) ? p : 0;
    for (int k = kbeg; k <= kend; ++k)
        for (int j = 1; j <= p; ++j)
            for (int i = 1; i <= p; ++i) {
                const int c[3] = {i, j, k};
                const double *qc = Pin + ora_vol(p, dim, i, j, k, nq);
                double D[ORA_MAXQ];
                for (int n = 0; n < dim; ++n) {
                    int lo[3] = {c[0], c[1], c[2]}, hi[3] = {c[0], c[1], c[2]};
                    lo[n] = c[n] - 1;
                    hi[n] = c[n] + 1;
                    const double *ql = Pin + ora_vol(p, dim, lo[0], lo[1], lo[2], nq);
                    const double *qh = Pin + ora_vol(p, dim, hi[0], hi[1], hi[2], nq);
                    double lp[ORA_MAXQ], lm[ORA_MAXQ], rp[ORA_MAXQ], rm[ORA_MAXQ];
                    ora_pde_face(P, ql, qc, n, prm, lp, lm);  /* face c - e_n/2 */
                    ora_pde_face(P, qc, qh, n, prm, rp, rm);  /* face c + e_n/2 */
                    for (int q = 0; q < P->nv; ++q) {
                        double d = lp[q] - rm[q];
                        if (n == 0) D[q] = d;
                        else D[q] = D[q] + d;
                    }
                }
                double *qo = Pout + ora_vol(p, dim, i, j, k, nq);
                double s[ORA_MAXQ];
                if (P->source) P->source(qc, prm, s);
                for (int q = 0; q < P->nv; ++q) {
                    double v = qc[q] + ratio * D[q];
                    qo[q] = P->source ? v + dt * s[q] : v;
                }
                for (int q = P->nv; q < nq; ++q) qo[q] = qc[q];
            }
}

static double ora_pde_patch_lambda(const ora_pde *P, const double *S, int p, int dim, const double *prm)
{
    double lmax = 0.0;
    int kbeg = (dim == 3) ? 1 : 0, kend = (dim == 3) ? p : 0;
    for (int k = kbeg; k <= kend; ++k)
        for (int j = 1; j <= p; ++j)
            for (int i = 1; i <= p; ++i)
                for (int n = 0; n < dim; ++n)
                    lmax = ora_max(lmax, P->eig(S + ora_vol(p, dim, i, j, k, P->nq), n, prm));
    return lmax;
}

/* Number of unknowns, evolved unknowns and parameters of a PDE in dim
 * dimensions; -1 if there is no such PDE. */
int fvo_pde_shape(int32_t pde, int32_t dim, int32_t *nq, int32_t *nv, int32_t *nprm)
{
    ora_pde P;
    int np = 0;
    if (ora_pde_get(pde, dim, &P, &np) != 0) return -1;
    *nq = P.nq;
    *nv = P.nv;
    *nprm = np;
    return 0;
}

/*
 * One explicit Euler step of every patch for the PDE `pde` (layout, periodic
 * and lambda_out as in fvo_batch_update; the unknowns per volume are the
 * PDE's).  prm holds nprm parameters.  Returns -1 for arguments the oracle
 * does not cover.  Serial (the acoustic PDEs keep their dimension in a
 * file-scope variable).
 */
int fvo_pde_update(int32_t pde, const double *prm, int32_t nprm, const double *in, double *out,
                   const int32_t *sizes, const int64_t *offsets, int32_t num_patches, int32_t dim,
                   double dt, double h, int32_t periodic, double *lambda_out)
{
    ora_pde P;
    int np = 0;
    if (ora_pde_get(pde, dim, &P, &np) != 0 || nprm < np || num_patches < 0) return -1;
    for (int32_t t = 0; t < num_patches; ++t) {
        int p = sizes[t];
        const double *Pin = in + offsets[t];
        double *Pout = out + offsets[t];
        ora_pde_patch_step(&P, Pin, Pout, p, dim, dt, h, prm);
        if (periodic) ora_wrap_faces(Pout, p, dim, P.nq);
        if (lambda_out) lambda_out[t] = ora_pde_patch_lambda(&P, Pout, p, dim, prm);
    }
    return 0;
}

/*
 * The user terms of one volume, for tests: f = F_n(q) (zeros without a flux),
 * lam = lambda_max,n(q), b = B_n(q) dq (zeros without a non-conservative
 * term), s = S(q) (zeros without a source); f, b, s over the evolved unknowns.
 */
int fvo_pde_terms(int32_t pde, int32_t dim, const double *prm, const double *q, int32_t n, const double *dq,
                  double *f, double *lam, double *b, double *s)
{
    ora_pde P;
    int np = 0;
    if (ora_pde_get(pde, dim, &P, &np) != 0 || n < 0 || n >= dim) return -1;
    for (int k = 0; k < P.nv; ++k) f[k] = b[k] = s[k] = 0.0;
    if (P.flux) P.flux(q, n, prm, f);
    *lam = P.eig(q, n, prm);
    if (P.ncp) P.ncp(q, dq, n, prm, b);
    if (P.source) P.source(q, prm, s);
    return 0;
}
