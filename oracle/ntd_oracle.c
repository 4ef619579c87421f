/*
 * ntd_oracle.c -- plain FP64 CPU oracle of the nested, twisted frequency-
 * filtering preconditioner ("NTD") of Aggarwal, Kakkar and Kumar,
 * "Multithreaded Filtering Preconditioner for Diffusion Equation on Structured
 * Grid", arXiv:1909.09771.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline of the benchmark load this library; the GPU library never does and
 * shares no code, header or table with it.  Single thread, no blocking, no
 * fusion, double precision, built with -ffp-contract=off.
 *
 * Grid (Sec. 2): nx points per line (x, fastest), ny lines per plane, nz
 * planes; unknown p = i + nx*(j + ny*k); nxy = nx*ny.  Every array has N =
 * nx*ny*nz entries.  Bands of a symmetric 7-point matrix: d (diagonal), ax
 * (coupling p <-> p+1, zero at i = nx-1), ay (p <-> p+nx, zero at j = ny-1),
 * az (p <-> p+nxy, zero at k = nz-1) -- the zero-padded band storage of Sec. 2.1.
 *
 * Twist ("meeting") block of a chain of nb blocks, 0-based: floor((nb-1)/2),
 * as in the LowerSolve / UpperSolve algorithms of Sec. 2.2.
 *
 * Readings of the paper taken here (the paper is silent or garbled there):
 *  - stencil: face coefficient = harmonic mean 2 k_p k_q / (k_p + k_q); a
 *    Dirichlet face adds k_p to the diagonal (ghost value 0 one step away),
 *    a Neumann face adds nothing; no h^2 factor.
 *  - the beta of a neighbour block nb of block k is (Pt_nb^{-1} w) ./ w with
 *    w = (coupling) .* t_k, where Pt_nb^{-1} is the nested (approximate) solve
 *    with block nb that the preconditioner itself applies; t is any positive
 *    filter vector (the paper uses t = 1).
 *  - level 3 adds a diagonal filter compensation (mode ORC_NEWTON_FILTERED)
 *    so that B t = A t holds exactly although the inner plane solve is only
 *    approximate; ORC_PAPER_LITERAL leaves it out, ORC_DIAG uses the
 *    classical diagonal beta instead of the Newton block 2b - bPb.
 *  - recurrences ending at "nz" at levels 2 and 1 are read as ending at ny, nx.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2
#define ORC_ENOTSPD 3
#define ORC_EBREAKDOWN 4
#define ORC_ENOCONV 5

#define ORC_NEWTON_FILTERED 0
#define ORC_PAPER_LITERAL 1
#define ORC_DIAG 2

#define BC_DIRICHLET 0

static int twist_index(int nb) { return (nb - 1) / 2; }

/* ------------------------------------------------------------------------- */
/* Assembly of A (Sec. 1, eq. diffeqn; structure of Sec. 2).                  */
/* ------------------------------------------------------------------------- */

static double face_coef(double kp, double kq) { return 2.0 * kp * kq / (kp + kq); }

int orc_assemble(int nx, int ny, int nz, const double *kappa, const int *bc,
                 double *d, double *ax, double *ay, double *az)
{
    if (nx < 1 || ny < 1 || nz < 1) return ORC_EINVAL;
    const long sx = 1, sy = nx, sz = (long)nx * ny;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long p = i + sy * j + sz * k;
                double kp = kappa[p];
                double diag = 0.0;
                /* faces in the order x-, x+, y-, y+, z-, z+ */
                if (i > 0) diag += face_coef(kp, kappa[p - sx]);
                else if (bc[0] == BC_DIRICHLET) diag += kp;
                if (i < nx - 1) { double c = face_coef(kp, kappa[p + sx]); diag += c; ax[p] = -c; }
                else { ax[p] = 0.0; if (bc[1] == BC_DIRICHLET) diag += kp; }
                if (j > 0) diag += face_coef(kp, kappa[p - sy]);
                else if (bc[2] == BC_DIRICHLET) diag += kp;
                if (j < ny - 1) { double c = face_coef(kp, kappa[p + sy]); diag += c; ay[p] = -c; }
                else { ay[p] = 0.0; if (bc[3] == BC_DIRICHLET) diag += kp; }
                if (k > 0) diag += face_coef(kp, kappa[p - sz]);
                else if (bc[4] == BC_DIRICHLET) diag += kp;
                if (k < nz - 1) { double c = face_coef(kp, kappa[p + sz]); diag += c; az[p] = -c; }
                else { az[p] = 0.0; if (bc[5] == BC_DIRICHLET) diag += kp; }
                d[p] = diag;
            }
    return ORC_OK;
}

/* y = A x from the four bands (7-point, symmetric). */
void orc_spmv(int nx, int ny, int nz, const double *d, const double *ax, const double *ay,
              const double *az, const double *x, double *y)
{
    const long sy = nx, sz = (long)nx * ny;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long p = i + sy * j + sz * k;
                double s = d[p] * x[p];
                if (i > 0) s += ax[p - 1] * x[p - 1];
                if (i < nx - 1) s += ax[p] * x[p + 1];
                if (j > 0) s += ay[p - sy] * x[p - sy];
                if (j < ny - 1) s += ay[p] * x[p + sy];
                if (k > 0) s += az[p - sz] * x[p - sz];
                if (k < nz - 1) s += az[p] * x[p + sz];
                y[p] = s;
            }
}

/* Neumaier-compensated dot product: the "exact" side of reduction checks. */
double orc_dot(long n, const double *x, const double *y)
{
    double s = 0.0, c = 0.0;
    for (long i = 0; i < n; ++i) {
        double v = x[i] * y[i];
        double t = s + v;
        if (fabs(s) >= fabs(v)) c += (s - t) + v;
        else c += (v - t) + s;
        s = t;
    }
    return s + c;
}

/* ------------------------------------------------------------------------- */
/* Level 1: exact twisted factorization of a tridiagonal line block           */
/* T = (M + L1)(I + M^{-1} U1)  (Sec. 2.1, recurrence for M_i).               */
/* ------------------------------------------------------------------------- */

/* Twisted pivots of the tridiagonal (d, e): e[i] couples i and i+1.
 * Returns ORC_ENOTSPD if a pivot is not positive and finite. */
static int line_pivots(int n, const double *d, const double *e, double *M)
{
    int j = twist_index(n);
    for (int i = 0; i < j; ++i)                    /* from the first row down */
        M[i] = (i == 0) ? d[0] : d[i] - e[i - 1] * e[i - 1] / M[i - 1];
    for (int i = n - 1; i > j; --i)                /* from the last row up */
        M[i] = (i == n - 1) ? d[n - 1] : d[i] - e[i] * e[i] / M[i + 1];
    double mj = d[j];                              /* the meeting row takes both */
    if (j > 0) mj -= e[j - 1] * e[j - 1] / M[j - 1];
    if (j < n - 1) mj -= e[j] * e[j] / M[j + 1];
    M[j] = mj;
    for (int i = 0; i < n; ++i)
        if (!(M[i] > 0.0) || !isfinite(M[i])) return ORC_ENOTSPD;
    return ORC_OK;
}

/* x = T^{-1} y with T = (M + L1)(I + M^{-1} U1): forward sweeps inward from both
 * ends to the twist row, then the twisted back substitution outward. g is
 * scratch of length n; x may alias y. */
static void line_solve(int n, const double *e, const double *M, const double *y,
                       double *x, double *g)
{
    int j = twist_index(n);
    for (int i = 0; i < j; ++i)
        g[i] = (y[i] - (i > 0 ? e[i - 1] * g[i - 1] : 0.0)) / M[i];
    for (int i = n - 1; i > j; --i)
        g[i] = (y[i] - (i < n - 1 ? e[i] * g[i + 1] : 0.0)) / M[i];
    double s = y[j];
    if (j > 0) s -= e[j - 1] * g[j - 1];
    if (j < n - 1) s -= e[j] * g[j + 1];
    g[j] = s / M[j];
    x[j] = g[j];
    for (int i = j - 1; i >= 0; --i) x[i] = g[i] - (e[i] / M[i]) * x[i + 1];
    for (int i = j + 1; i < n; ++i) x[i] = g[i] - (e[i - 1] / M[i]) * x[i - 1];
}

/* ------------------------------------------------------------------------- */
/* The nested solve B^{-1} (Sec. 2.2, Algorithms 1-7), 0-based, recursive     */
/* over the three levels: level 3 = planes coupled by g3 (= az), level 2 =    */
/* lines of a plane coupled by f2 (the y-band of P), level 1 = line solves.   */
/* ------------------------------------------------------------------------- */

typedef struct {
    int nx, ny, nz;
    const double *e1, *M, *f2, *g3;
    double *tmp[4], *cor[4]; /* per-level scratch: right-hand side, correction of a block */
    double *g1;              /* level-1 scratch */
} solver;

/* block count, block size and coupling band of level 2 (lines) or 3 (planes) */
static void level_shape(const solver *S, int level, int *nb, long *bs, const double **band)
{
    if (level == 3) { *nb = S->nz; *bs = (long)S->nx * S->ny; *band = S->g3; }
    else { *nb = S->ny; *bs = S->nx; *band = S->f2; }
}

static void lower_sweep(solver *S, int level, long fbase, double *x, const double *b);
static void upper_sweep(solver *S, int level, long fbase, double *x);

/* SOLVE of Algorithm 1: x = (block of B at `level` whose first unknown is
 * fbase)^{-1} b, with x and b indexed relative to the block.  Level 1 is the
 * exact line solve; levels 2 and 3 are a lower then an upper twisted sweep. */
static void nested_solve(solver *S, int level, long fbase, double *x, const double *b)
{
    if (level == 1) {
        line_solve(S->nx, S->e1 + fbase, S->M + fbase, b, x, S->g1);
        return;
    }
    lower_sweep(S, level, fbase, x, b);
    upper_sweep(S, level, fbase, x);
}

/* (Pt + L) w = b, the twisted block lower sweep (Algs 2-4): sub-blocks above
 * the twist are solved top-down, those below bottom-up, the twist block last
 * with both neighbours.  band[q*bs + u] couples sub-blocks q and q+1. */
static void lower_sweep(solver *S, int level, long fbase, double *x, const double *b)
{
    int nb; long bs; const double *band;
    level_shape(S, level, &nb, &bs, &band);
    const double *L = band + fbase;
    int jt = twist_index(nb);
    double *t = S->tmp[level];
    for (int q = 0; q < jt; ++q) {
        long s = q * bs;
        for (long u = 0; u < bs; ++u)
            t[u] = b[s + u] - (q > 0 ? L[s - bs + u] * x[s - bs + u] : 0.0);
        nested_solve(S, level - 1, fbase + s, x + s, t);
    }
    for (int q = nb - 1; q > jt; --q) {
        long s = q * bs;
        for (long u = 0; u < bs; ++u)
            t[u] = b[s + u] - (q < nb - 1 ? L[s + u] * x[s + bs + u] : 0.0);
        nested_solve(S, level - 1, fbase + s, x + s, t);
    }
    long s = jt * bs;
    for (long u = 0; u < bs; ++u) {
        double v = b[s + u];
        if (jt > 0) v -= L[s - bs + u] * x[s - bs + u];
        if (jt < nb - 1) v -= L[s + u] * x[s + bs + u];
        t[u] = v;
    }
    nested_solve(S, level - 1, fbase + s, x + s, t);
}

/* (I + Pt^{-1} U) x = w, in place on x = w (Algs 5-7): the twist block keeps
 * w; going outward, each sub-block subtracts its solve applied to U times the
 * already final neighbour toward the twist. */
static void upper_sweep(solver *S, int level, long fbase, double *x)
{
    int nb; long bs; const double *band;
    level_shape(S, level, &nb, &bs, &band);
    const double *U = band + fbase;
    int jt = twist_index(nb);
    double *t = S->tmp[level], *c = S->cor[level];
    for (int q = jt - 1; q >= 0; --q) {
        long s = q * bs;
        for (long u = 0; u < bs; ++u) t[u] = U[s + u] * x[s + bs + u];
        nested_solve(S, level - 1, fbase + s, c, t);
        for (long u = 0; u < bs; ++u) x[s + u] -= c[u];
    }
    for (int q = jt + 1; q < nb; ++q) {
        long s = q * bs;
        for (long u = 0; u < bs; ++u) t[u] = U[s - bs + u] * x[s - bs + u];
        nested_solve(S, level - 1, fbase + s, c, t);
        for (long u = 0; u < bs; ++u) x[s + u] -= c[u];
    }
}

static int solver_init(solver *S, int nx, int ny, int nz, const double *e1, const double *M,
                       const double *f2, const double *g3)
{
    memset(S, 0, sizeof(*S));
    S->nx = nx; S->ny = ny; S->nz = nz;
    S->e1 = e1; S->M = M; S->f2 = f2; S->g3 = g3;
    long nxy = (long)nx * ny;
    S->tmp[3] = malloc(sizeof(double) * nxy); S->cor[3] = malloc(sizeof(double) * nxy);
    S->tmp[2] = malloc(sizeof(double) * nx);  S->cor[2] = malloc(sizeof(double) * nx);
    S->g1 = malloc(sizeof(double) * nx);
    if (!S->tmp[3] || !S->cor[3] || !S->tmp[2] || !S->cor[2] || !S->g1) return ORC_ENOMEM;
    return ORC_OK;
}

static void solver_free(solver *S)
{
    free(S->tmp[3]); free(S->cor[3]); free(S->tmp[2]); free(S->cor[2]); free(S->g1);
}

/* z = B^{-1} r: SOLVE(whole vector, level 3) of Algorithm 1. */
int orc_apply(int nx, int ny, int nz, const double *e1, const double *M, const double *f2,
              const double *g3, const double *r, double *z)
{
    solver S;
    if (solver_init(&S, nx, ny, nz, e1, M, f2, g3) != ORC_OK) { solver_free(&S); return ORC_ENOMEM; }
    nested_solve(&S, 3, 0, z, r);
    solver_free(&S);
    return ORC_OK;
}

/* x = Pt_k^{-1} y for the single plane k (level-2 solve with plane k's factors). */
int orc_plane_solve(int nx, int ny, int nz, const double *e1, const double *M, const double *f2,
                    int k, const double *y, double *x)
{
    solver S;
    if (k < 0 || k >= nz) return ORC_EINVAL;
    if (solver_init(&S, nx, ny, nz, e1, M, f2, NULL) != ORC_OK) { solver_free(&S); return ORC_ENOMEM; }
    nested_solve(&S, 2, (long)k * nx * ny, x, y);
    solver_free(&S);
    return ORC_OK;
}

/* x = T^{-1} y for one tridiagonal (d unused by the solve; pivots M given). */
void orc_line_solve(int n, const double *e, const double *M, const double *y, double *x)
{
    double *g = malloc(sizeof(double) * (n > 0 ? n : 1));
    line_solve(n, e, M, y, x, g);
    free(g);
}

int orc_line_pivots(int n, const double *d, const double *e, double *M)
{
    return line_pivots(n, d, e, M);
}

/* ------------------------------------------------------------------------- */
/* Setup (Sec. 2.1): level-3 recurrence for the plane blocks P_k, level-2     */
/* recurrence for the line blocks T_m of each P_k, level-1 twisted pivots.    */
/* ------------------------------------------------------------------------- */

typedef struct {
    int nx, ny, nz, mode;
    const double *d, *ax, *ay, *az, *t;
    /* P's bands: dP (diagonal), xP (x-band), f2 (y-band) ; T's bands: dT, e1 ; pivots M */
    double *dP, *xP, *f2, *dT, *e1, *M;
    double *w, *z, *beta, *Pz; /* plane scratch */
    double *v, *zl, *gam;      /* line scratch */
    solver S;
} builder;

/* Line m of plane k: T_m starts as the line block of P_k and loses, for each
 * neighbour line nb, phi (2 g - g T_nb g) phi with g = diag((T_nb^{-1} v) ./ v),
 * v = phi .* t_m, phi = the y-coupling between the two lines (Sec. 2.1, T_i
 * recurrence); then its twisted pivots. */
static int build_line(builder *Bd, int k, int m, int nnb, const int *nbs)
{
    const int nx = Bd->nx;
    const long nxy = (long)nx * Bd->ny;
    const long lm = (long)k * nxy + (long)m * nx;
    for (int i = 0; i < nx; ++i) { Bd->dT[lm + i] = Bd->dP[lm + i]; Bd->e1[lm + i] = Bd->xP[lm + i]; }
    for (int a = 0; a < nnb; ++a) {
        int nb = nbs[a];
        long ln = (long)k * nxy + (long)nb * nx;
        long lc = (long)k * nxy + (long)(m < nb ? m : nb) * nx; /* coupling stored on the lower line */
        const double *phi = Bd->f2 + lc;
        for (int i = 0; i < nx; ++i) Bd->v[i] = phi[i] * Bd->t[lm + i];
        line_solve(nx, Bd->e1 + ln, Bd->M + ln, Bd->v, Bd->zl, Bd->S.g1);
        for (int i = 0; i < nx; ++i) Bd->gam[i] = Bd->zl[i] / Bd->v[i];
        if (Bd->mode == ORC_DIAG) {
            for (int i = 0; i < nx; ++i) Bd->dT[lm + i] -= phi[i] * phi[i] * Bd->gam[i];
        } else {
            for (int i = 0; i < nx; ++i) {
                double g = Bd->gam[i];
                double yii = 2.0 * g - g * Bd->dT[ln + i] * g;
                Bd->dT[lm + i] -= phi[i] * yii * phi[i];
            }
            for (int i = 0; i + 1 < nx; ++i) {
                double yi1 = -Bd->gam[i] * Bd->e1[ln + i] * Bd->gam[i + 1];
                Bd->e1[lm + i] -= phi[i] * yi1 * phi[i + 1];
            }
        }
    }
    return line_pivots(nx, Bd->dT + lm, Bd->e1 + lm, Bd->M + lm);
}

/* Level-2 factorization P_k = (T + L2)(I + T^{-1} U2) of plane k. */
static int build_plane_lines(builder *Bd, int k)
{
    const int ny = Bd->ny;
    int jt = twist_index(ny), st, nbs[2] = {0, 0};
    for (int m = 0; m < jt; ++m) {
        int n = 0; if (m > 0) nbs[n++] = m - 1;
        if ((st = build_line(Bd, k, m, n, nbs)) != ORC_OK) return st;
    }
    for (int m = ny - 1; m > jt; --m) {
        int n = 0; if (m < ny - 1) nbs[n++] = m + 1;
        if ((st = build_line(Bd, k, m, n, nbs)) != ORC_OK) return st;
    }
    int n = 0;
    if (jt > 0) nbs[n++] = jt - 1;
    if (jt < ny - 1) nbs[n++] = jt + 1;
    return build_line(Bd, k, jt, n, nbs);
}

/* Plane k: P_k starts as D^_k and loses, for each neighbour plane nb,
 * psi (2 b - b P_nb b) psi with b = diag((Pt_nb^{-1} w) ./ w), w = psi .* t_k,
 * psi = the z-coupling (Sec. 2.1, approximate P_i recurrence); in the filtered
 * mode the diagonal then gains psi b (w - P_nb z) ./ t_k.  Then level 2. */
static int build_plane(builder *Bd, int k, int nnb, const int *nbs)
{
    const int nx = Bd->nx, ny = Bd->ny;
    const long nxy = (long)nx * ny, pk = (long)k * nxy;
    for (long u = 0; u < nxy; ++u) {
        Bd->dP[pk + u] = Bd->d[pk + u];
        Bd->xP[pk + u] = Bd->ax[pk + u];
        Bd->f2[pk + u] = Bd->ay[pk + u];
    }
    for (int a = 0; a < nnb; ++a) {
        int nb = nbs[a];
        long pn = (long)nb * nxy;
        const double *psi = Bd->az + (long)(k < nb ? k : nb) * nxy;
        for (long u = 0; u < nxy; ++u) Bd->w[u] = psi[u] * Bd->t[pk + u];
        nested_solve(&Bd->S, 2, pn, Bd->z, Bd->w);
        for (long u = 0; u < nxy; ++u) Bd->beta[u] = Bd->z[u] / Bd->w[u];
        const double *dPn = Bd->dP + pn, *xPn = Bd->xP + pn, *yPn = Bd->f2 + pn;
        if (Bd->mode == ORC_DIAG) {
            for (long u = 0; u < nxy; ++u) Bd->dP[pk + u] -= psi[u] * psi[u] * Bd->beta[u];
            continue;
        }
        /* P_nb z on the plane (5-point), needed by the compensation */
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long u = i + (long)nx * j;
                double s = dPn[u] * Bd->z[u];
                if (i > 0) s += xPn[u - 1] * Bd->z[u - 1];
                if (i < nx - 1) s += xPn[u] * Bd->z[u + 1];
                if (j > 0) s += yPn[u - nx] * Bd->z[u - nx];
                if (j < ny - 1) s += yPn[u] * Bd->z[u + nx];
                Bd->Pz[u] = s;
            }
        for (long u = 0; u < nxy; ++u) {
            double b = Bd->beta[u];
            double xuu = 2.0 * b - b * dPn[u] * b;
            Bd->dP[pk + u] -= psi[u] * xuu * psi[u];
        }
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long u = i + (long)nx * j;
                if (i < nx - 1) {
                    double x01 = -Bd->beta[u] * xPn[u] * Bd->beta[u + 1];
                    Bd->xP[pk + u] -= psi[u] * x01 * psi[u + 1];
                }
                if (j < ny - 1) {
                    double x0n = -Bd->beta[u] * yPn[u] * Bd->beta[u + nx];
                    Bd->f2[pk + u] -= psi[u] * x0n * psi[u + nx];
                }
            }
        if (Bd->mode == ORC_NEWTON_FILTERED)
            for (long u = 0; u < nxy; ++u)
                Bd->dP[pk + u] += psi[u] * Bd->beta[u] * (Bd->w[u] - Bd->Pz[u]) / Bd->t[pk + u];
    }
    return build_plane_lines(Bd, k);
}

/*
 * Factorization B = (Pt + L3)(I + Pt^{-1} U3) with Pt_k = (T + L2)(I + T^{-1} U2)
 * and T_m = (M + L1)(I + M^{-1} U1).
 * Inputs: the bands of A, the filter vector t (NULL = ones), the mode.
 * Outputs (length N each): e1 = x-band of T, M = twisted pivots of T,
 * f2 = y-band of P.  Optional outputs (NULL to skip): dT = diagonal of T,
 * dP = diagonal of P, xP = x-band of P.  The z-band used by the solve is az.
 */
int orc_setup(int nx, int ny, int nz, const double *d, const double *ax, const double *ay,
              const double *az, const double *t, int mode, double *e1, double *M, double *f2,
              double *dT, double *dP, double *xP)
{
    if (nx < 1 || ny < 1 || nz < 1) return ORC_EINVAL;
    if (mode != ORC_NEWTON_FILTERED && mode != ORC_PAPER_LITERAL && mode != ORC_DIAG) return ORC_EINVAL;
    const long N = (long)nx * ny * nz, nxy = (long)nx * ny;
    builder Bd;
    memset(&Bd, 0, sizeof(Bd));
    Bd.nx = nx; Bd.ny = ny; Bd.nz = nz; Bd.mode = mode;
    Bd.d = d; Bd.ax = ax; Bd.ay = ay; Bd.az = az;
    double *ones = NULL, *own_dT = NULL, *own_dP = NULL, *own_xP = NULL;
    if (!t) { ones = malloc(sizeof(double) * N); if (!ones) return ORC_ENOMEM; for (long p = 0; p < N; ++p) ones[p] = 1.0; t = ones; }
    Bd.t = t;
    Bd.e1 = e1; Bd.M = M; Bd.f2 = f2;
    Bd.dT = dT ? dT : (own_dT = malloc(sizeof(double) * N));
    Bd.dP = dP ? dP : (own_dP = malloc(sizeof(double) * N));
    Bd.xP = xP ? xP : (own_xP = malloc(sizeof(double) * N));
    Bd.w = malloc(sizeof(double) * nxy); Bd.z = malloc(sizeof(double) * nxy);
    Bd.beta = malloc(sizeof(double) * nxy); Bd.Pz = malloc(sizeof(double) * nxy);
    Bd.v = malloc(sizeof(double) * nx); Bd.zl = malloc(sizeof(double) * nx); Bd.gam = malloc(sizeof(double) * nx);
    int st = solver_init(&Bd.S, nx, ny, nz, e1, M, f2, az);
    if (st == ORC_OK && (!Bd.dT || !Bd.dP || !Bd.xP || !Bd.w || !Bd.z || !Bd.beta || !Bd.Pz ||
                         !Bd.v || !Bd.zl || !Bd.gam)) st = ORC_ENOMEM;
    if (st == ORC_OK) {
        int jt = twist_index(nz), nbs[2] = {0, 0};
        for (int k = 0; k < jt && st == ORC_OK; ++k) {
            int n = 0; if (k > 0) nbs[n++] = k - 1;
            st = build_plane(&Bd, k, n, nbs);
        }
        for (int k = nz - 1; k > jt && st == ORC_OK; --k) {
            int n = 0; if (k < nz - 1) nbs[n++] = k + 1;
            st = build_plane(&Bd, k, n, nbs);
        }
        if (st == ORC_OK) {
            int n = 0;
            if (jt > 0) nbs[n++] = jt - 1;
            if (jt < nz - 1) nbs[n++] = jt + 1;
            st = build_plane(&Bd, jt, n, nbs);
        }
    }
    solver_free(&Bd.S);
    free(Bd.w); free(Bd.z); free(Bd.beta); free(Bd.Pz); free(Bd.v); free(Bd.zl); free(Bd.gam);
    free(own_dT); free(own_dP); free(own_xP); free(ones);
    return st;
}

/* ------------------------------------------------------------------------- */
/* ILU(0) smoother and the combination preconditioner (Sec. 3, "Smoothing     */
/* high frequency components of error", eq. com, and "Parallel Solve with     */
/* Preconditioner"): ILU(0) of the block-diagonal approximation               */
/* blkD(A(1:M,1:M), A(M+1:N,M+1:N)), M = floor(N/2) (nblocks = 2), or of A    */
/* itself (nblocks = 1).  For the 7-point pattern ILU(0) creates no fill      */
/* inside the pattern, so only the diagonal changes:                          */
/*   dt_p = a_pp - sum over kept lower neighbours q of a_pq^2 / dt_q,         */
/* and B_ILU = (Dt + L) Dt^{-1} (Dt + U) with L, U the kept strict parts.     */
/* ------------------------------------------------------------------------- */

/* Is the coupling between rows p < q kept by the block-diagonal split? */
static int ilu_kept(long p, long q, long M, int nblocks)
{
    return nblocks == 1 || !(p < M && q >= M);
}

int orc_ilu0(int nx, int ny, int nz, const double *d, const double *ax, const double *ay,
             const double *az, int nblocks, double *dt)
{
    if (nblocks != 1 && nblocks != 2) return ORC_EINVAL;
    const long sy = nx, sz = (long)nx * ny, N = sz * nz, M = N / 2;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long p = i + sy * j + sz * k;
                double v = d[p];
                if (i > 0 && ilu_kept(p - 1, p, M, nblocks)) v -= ax[p - 1] * ax[p - 1] / dt[p - 1];
                if (j > 0 && ilu_kept(p - sy, p, M, nblocks)) v -= ay[p - sy] * ay[p - sy] / dt[p - sy];
                if (k > 0 && ilu_kept(p - sz, p, M, nblocks)) v -= az[p - sz] * az[p - sz] / dt[p - sz];
                if (!(v > 0.0) || !isfinite(v)) return ORC_ENOTSPD;
                dt[p] = v;
            }
    return ORC_OK;
}

/* z = B_ILU^{-1} r: forward sweep (Dt + L) y = r, then (I + Dt^{-1} U) z = y. */
void orc_ilu0_apply(int nx, int ny, int nz, const double *ax, const double *ay, const double *az,
                    const double *dt, int nblocks, const double *r, double *z)
{
    const long sy = nx, sz = (long)nx * ny, N = sz * nz, M = N / 2;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                long p = i + sy * j + sz * k;
                double v = r[p];
                if (i > 0 && ilu_kept(p - 1, p, M, nblocks)) v -= ax[p - 1] * z[p - 1];
                if (j > 0 && ilu_kept(p - sy, p, M, nblocks)) v -= ay[p - sy] * z[p - sy];
                if (k > 0 && ilu_kept(p - sz, p, M, nblocks)) v -= az[p - sz] * z[p - sz];
                z[p] = v / dt[p];
            }
    for (int k = nz - 1; k >= 0; --k)
        for (int j = ny - 1; j >= 0; --j)
            for (int i = nx - 1; i >= 0; --i) {
                long p = i + sy * j + sz * k;
                double v = 0.0;
                if (i < nx - 1 && ilu_kept(p, p + 1, M, nblocks)) v += ax[p] * z[p + 1];
                if (j < ny - 1 && ilu_kept(p, p + sy, M, nblocks)) v += ay[p] * z[p + sy];
                if (k < nz - 1 && ilu_kept(p, p + sz, M, nblocks)) v += az[p] * z[p + sz];
                z[p] -= v / dt[p];
            }
}

/* The combination of eq. com, evaluated as written:
 * z = B^{-1} r + B_ILU^{-1} r - B^{-1} A B_ILU^{-1} r. */
int orc_combo_apply(int nx, int ny, int nz, const double *d, const double *ax, const double *ay,
                    const double *az, const double *e1, const double *M_, const double *f2,
                    const double *dt, int nblocks, const double *r, double *z)
{
    const long N = (long)nx * ny * nz;
    double *zi = malloc(sizeof(double) * N), *t = malloc(sizeof(double) * N);
    double *zb = malloc(sizeof(double) * N);
    if (!zi || !t || !zb) { free(zi); free(t); free(zb); return ORC_ENOMEM; }
    orc_apply(nx, ny, nz, e1, M_, f2, az, r, z);                  /* B^{-1} r */
    orc_ilu0_apply(nx, ny, nz, ax, ay, az, dt, nblocks, r, zi);    /* B_ILU^{-1} r */
    orc_spmv(nx, ny, nz, d, ax, ay, az, zi, t);                   /* A B_ILU^{-1} r */
    orc_apply(nx, ny, nz, e1, M_, f2, az, t, zb);                 /* B^{-1} A B_ILU^{-1} r */
    for (long p = 0; p < N; ++p) z[p] = z[p] + zi[p] - zb[p];
    free(zi); free(t); free(zb);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Preconditioned conjugate gradient (Sec. 1; stopping rule of Sec. 3):       */
/* x0 = 0, stop when ||r||/||b|| <= tol on the recursively updated residual,  */
/* then confirm with the true residual ||b - A x||/||b|| (iterate on if it is */
/* still above tol).  iters counts products with A inside the loop.  With dt  */
/* (ILU(0) diagonal, nblocks blocks) the preconditioner is the combination.   */
/* CG needs p'Ap > 0 (A positive definite) and r'z > 0 (a positive definite   */
/* preconditioner); the combination of eq. com is not symmetric, so r'z can   */
/* turn non-positive.  Either one ends the loop with ORC_EBREAKDOWN, x being  */
/* the last iterate.                                                          */
/* ------------------------------------------------------------------------- */
/* The symmetric combination (an addition to the paper, whose eq. com is not
 * symmetric), its three steps in order:
 *   z1 = B_ILU^{-1} r,  z2 = z1 + B^{-1} (r - A z1),  z = z2 + B_ILU^{-1} (r - A z2). */
int orc_sym_combo_apply(int nx, int ny, int nz, const double *d, const double *ax,
                        const double *ay, const double *az, const double *e1, const double *M_,
                        const double *f2, const double *dt, int nblocks, const double *r,
                        double *z)
{
    const long N = (long)nx * ny * nz;
    double *t = malloc(sizeof(double) * N), *u = malloc(sizeof(double) * N);
    if (!t || !u) { free(t); free(u); return ORC_ENOMEM; }
    orc_ilu0_apply(nx, ny, nz, ax, ay, az, dt, nblocks, r, z);      /* z = z1 */
    orc_spmv(nx, ny, nz, d, ax, ay, az, z, t);
    for (long p = 0; p < N; ++p) t[p] = r[p] - t[p];                 /* r - A z1 */
    orc_apply(nx, ny, nz, e1, M_, f2, az, t, u);
    for (long p = 0; p < N; ++p) z[p] += u[p];                       /* z = z2 */
    orc_spmv(nx, ny, nz, d, ax, ay, az, z, t);
    for (long p = 0; p < N; ++p) t[p] = r[p] - t[p];                 /* r - A z2 */
    orc_ilu0_apply(nx, ny, nz, ax, ay, az, dt, nblocks, t, u);
    for (long p = 0; p < N; ++p) z[p] += u[p];
    free(t); free(u);
    return ORC_OK;
}

/* Preconditioner of the PCG: B^{-1} (combo 0), the combination of eq. com
 * (combo 1) or the symmetric combination (combo 2); dt is the ILU(0) diagonal. */
static void pcg_precond(int nx, int ny, int nz, const double *d, const double *ax,
                        const double *ay, const double *az, const double *e1, const double *M,
                        const double *f2, const double *dt, int nblocks, int combo,
                        const double *r, double *z)
{
    if (combo == 2) orc_sym_combo_apply(nx, ny, nz, d, ax, ay, az, e1, M, f2, dt, nblocks, r, z);
    else if (combo == 1) orc_combo_apply(nx, ny, nz, d, ax, ay, az, e1, M, f2, dt, nblocks, r, z);
    else orc_apply(nx, ny, nz, e1, M, f2, az, r, z);
}

int orc_pcg_combo(int nx, int ny, int nz, const double *d, const double *ax, const double *ay,
                  const double *az, const double *e1, const double *M, const double *f2,
                  const double *dt, int nblocks, int combo, const double *b, double *x,
                  double tol, int maxit, int *iters, double *relres, double *hist)
{
    if (combo < 0 || combo > 2 || (combo > 0 && !dt)) return ORC_EINVAL;
    const long N = (long)nx * ny * nz;
    double *r = malloc(sizeof(double) * N), *z = malloc(sizeof(double) * N);
    double *p = malloc(sizeof(double) * N), *q = malloc(sizeof(double) * N);
    int st = ORC_OK;
    if (!r || !z || !p || !q) { st = ORC_ENOMEM; goto done; }
    double bn = sqrt(orc_dot(N, b, b));
    for (long i = 0; i < N; ++i) { x[i] = 0.0; r[i] = b[i]; }
    *iters = 0;
    if (bn == 0.0) { *relres = 0.0; goto done; }
    pcg_precond(nx, ny, nz, d, ax, ay, az, e1, M, f2, dt, nblocks, combo, r, z);
    for (long i = 0; i < N; ++i) p[i] = z[i];
    double rho = orc_dot(N, r, z);
    int it = 0;
    if (!(rho > 0.0) || !isfinite(rho)) st = ORC_EBREAKDOWN;
    while (st == ORC_OK) {
        if (it >= maxit) { st = ORC_ENOCONV; break; }
        orc_spmv(nx, ny, nz, d, ax, ay, az, p, q);
        double pq = orc_dot(N, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { st = ORC_EBREAKDOWN; break; }
        double alpha = rho / pq;
        for (long i = 0; i < N; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        ++it;
        double rn = sqrt(orc_dot(N, r, r)) / bn;
        if (hist) hist[it - 1] = rn;
        if (rn <= tol) {
            orc_spmv(nx, ny, nz, d, ax, ay, az, x, q);  /* true residual check */
            for (long i = 0; i < N; ++i) q[i] = b[i] - q[i];
            double tr = sqrt(orc_dot(N, q, q)) / bn;
            if (tr <= tol) break;
        }
        pcg_precond(nx, ny, nz, d, ax, ay, az, e1, M, f2, dt, nblocks, combo, r, z);
        double rho_new = orc_dot(N, r, z);
        if (!(rho_new > 0.0) || !isfinite(rho_new)) { st = ORC_EBREAKDOWN; break; }
        double beta = rho_new / rho;
        rho = rho_new;
        for (long i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
    }
    *iters = it;
    orc_spmv(nx, ny, nz, d, ax, ay, az, x, q);
    for (long i = 0; i < N; ++i) q[i] = b[i] - q[i];
    *relres = sqrt(orc_dot(N, q, q)) / bn;
done:
    free(r); free(z); free(p); free(q);
    return st;
}

/* PCG with B^{-1} (dt == NULL) or with the combination of eq. com (dt given). */
int orc_pcg(int nx, int ny, int nz, const double *d, const double *ax, const double *ay,
            const double *az, const double *e1, const double *M, const double *f2,
            const double *dt, int nblocks, const double *b, double *x, double tol, int maxit,
            int *iters, double *relres, double *hist)
{
    return orc_pcg_combo(nx, ny, nz, d, ax, ay, az, e1, M, f2, dt, nblocks, dt ? 1 : 0, b, x, tol,
                         maxit, iters, relres, hist);
}
