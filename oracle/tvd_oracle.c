/*
 * Plain FP64 CPU oracle for one step of GAMER's dimensionally split relaxing
 * TVD scheme (Schive, Tsai & Chiueh, "GAMER: a GPU-Accelerated Adaptive Mesh
 * Refinement Code for Astrophysics", Sec. 2.2) on cubic blocks of cells that
 * carry three ghost zones on every side.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the HIP path is checked against.  It shares no code, header,
 * table or helper with the HIP path, and nothing on the product path may call
 * it.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it.
 *
 * Every routine follows the paper's steps in the paper's order:
 *   Eqs. (ThermalEnergy), (EOS)   pressure from the conserved variables
 *   Eq.  (1DEuler), Sec. 2.2      freezing speed c = |v| + c_s
 *   Eq.  (LRFlux)                 right/left moving fluxes F^R, F^L
 *   Eq.  (MidpointValue)          first-order upwind half step
 *   Eqs. (2ndTVDFluxCorr), (2ndFluxCorr), (vanLeer), (2ndRFlux)
 *                                 second-order limited interface fluxes
 *   Eq.  (FullstepValue)          full step from u^t with the midpoint fluxes
 *   Sec. 2.2 (last paragraphs)    dimensional splitting, forward xyz /
 *                                 backward zyx, seven-point stencil, three
 *                                 ghost zones
 *   Eq.  (CFL), Sec. 3.4          maximum signal speed for the time step
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes):
 *   - F^R = (c u + F)/2, F^L = (c u - F)/2: the paper's c (u +/- w)/2 with
 *     w = F/c, multiplied out so that c = 0 needs no division.
 *   - 3-D flux: five components, transverse momenta advected by v_d.
 *   - kinetic energy summed as (m_d v_d + (m_t1 v_t1 + m_t2 v_t2))/2.
 *   - freezing speed per cell and per sweep: c = |v_d| + c_s, recomputed from
 *     the midpoint state.
 *   - pressure floor P* = max(P, p_floor) inside fluxes, sound speed and the
 *     signal speed only; the stored energy is never modified.
 *   - the left-moving limited flux is the mirror image of Eq. (2ndRFlux)
 *     about the interface.
 *   - region rule: within one step the sweep along d updates cells whose
 *     transverse coordinates lie in [-3, n+3) along axes swept later in the
 *     step and in [0, n) along axes swept earlier.
 *
 * Layout of a block: five consecutive cubes (rho, m_x, m_y, m_z, e), each
 * (n+6)^3 doubles with x fastest, then y, then z.  Output blocks hold the
 * n^3 interior cells in the same variable and axis order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NVAR 5
#define GHOST 3
#define PATCH 8   /* patch edge: boundary fluxes are kept at multiples of it */

/* ---------------------------------------------------------------------- */
/* Cell level: Eqs. (ThermalEnergy), (EOS), (LRFlux)                        */
/* ---------------------------------------------------------------------- */

/* Pressure floor rule: P* = P unless P < p_floor.  Counts floored cells and
 * cells with non-positive density. */
typedef struct {
    long long floored;
    long long nonphysical;
} oracle_counts;

/*
 * Right- and left-moving fluxes of one cell for a sweep along axis d
 * (0 = x, 1 = y, 2 = z).  u and the outputs use the global component order
 * (rho, m_x, m_y, m_z, e).  Returns the freezing speed c.
 */
double oracle_split_fluxes(const double u[NVAR], int d, double gamma,
                           double p_floor, double FR[NVAR], double FL[NVAR],
                           oracle_counts *cnt)
{
    const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    const double rho = u[0];
    const double m_d = u[1 + d], m_t1 = u[1 + t1], m_t2 = u[1 + t2];
    const double e = u[4];

    if (cnt && !(rho > 0.0)) cnt->nonphysical++;

    /* velocities */
    const double v_d = m_d / rho;
    const double v_t1 = m_t1 / rho;
    const double v_t2 = m_t2 / rho;

    /* Eq. (ThermalEnergy): e = rho v^2 / 2 + eps;  Eq. (EOS): P = (gamma-1) eps */
    const double kin = 0.5 * (m_d * v_d + (m_t1 * v_t1 + m_t2 * v_t2));
    double P = (gamma - 1.0) * (e - kin);
    if (P < p_floor) {
        if (cnt) cnt->floored++;
        P = p_floor;
    }

    /* freezing speed c = |v| + c_s with c_s = sqrt(gamma P / rho) */
    const double cs = sqrt(gamma * P / rho);
    const double c = fabs(v_d) + cs;

    /* flux vector F(u) along d: (rho v_d, rho v v_d + P delta, (e + P) v_d) */
    double F[NVAR];
    F[0] = m_d;
    F[1 + d] = m_d * v_d + P;
    F[1 + t1] = m_t1 * v_d;
    F[1 + t2] = m_t2 * v_d;
    F[4] = (e + P) * v_d;

    /* Eq. (LRFlux): F^R = c (u + w)/2, F^L = c (u - w)/2 with w = F/c */
    for (int k = 0; k < NVAR; ++k) {
        FR[k] = 0.5 * (c * u[k] + F[k]);
        FL[k] = 0.5 * (c * u[k] - F[k]);
    }
    return c;
}

/* Eq. (vanLeer): harmonic mean of the two flux corrections, zero at extrema. */
double oracle_vanleer(double dF1, double dF2)
{
    if (dF1 * dF2 > 0.0) return 2.0 * dF1 * dF2 / (dF1 + dF2);
    return 0.0;
}

/* ---------------------------------------------------------------------- */
/* Pencil level: the 1-D operator of Eqs. (MidpointValue)-(FullstepValue)  */
/* ---------------------------------------------------------------------- */

/*
 * Advance one pencil of n+6 cells (cells -3 .. n+2, stored at array index
 * i+3) along axis d by dt with zone size dh.  q holds (n+6) x 5 values in the
 * global component order; out receives the n updated interior cells.
 * hface, if not NULL, receives the (n+1) x 5 second-order interface fluxes
 * that the full step uses: row i is the flux through interface i-1/2 of
 * interior cell i (i = 0 .. n), so that out_i = q_i - dt/dh (row i+1 - row i).
 */
void oracle_pencil_flux(const double *q, int n, int d, double dt, double dh,
                        double gamma, double p_floor, double *out, double *hface,
                        oracle_counts *cnt)
{
    const int L = n + 2 * GHOST;

    double *FR = (double *)malloc(sizeof(double) * L * NVAR);
    double *FL = (double *)malloc(sizeof(double) * L * NVAR);
    double *G = (double *)malloc(sizeof(double) * L * NVAR);   /* G[j]: interface j+1/2 */
    double *h = (double *)malloc(sizeof(double) * L * NVAR);
    double *FRh = (double *)malloc(sizeof(double) * L * NVAR);
    double *FLh = (double *)malloc(sizeof(double) * L * NVAR);
    double *H = (double *)malloc(sizeof(double) * L * NVAR);   /* H[j]: interface j+1/2 */

    /* (1) freezing speed and split fluxes at time t, all cells */
    for (int j = 0; j < L; ++j)
        oracle_split_fluxes(q + j * NVAR, d, gamma, p_floor, FR + j * NVAR,
                            FL + j * NVAR, cnt);

    /* (2) first-order upwind interface flux, F_{j+1/2} = F^R_j - F^L_{j+1} */
    for (int j = 0; j + 1 < L; ++j)
        for (int k = 0; k < NVAR; ++k)
            G[j * NVAR + k] = FR[j * NVAR + k] - FL[(j + 1) * NVAR + k];

    /* (3) Eq. (MidpointValue): half step, cells j = 1 .. L-2 */
    for (int j = 1; j + 1 < L; ++j)
        for (int k = 0; k < NVAR; ++k)
            h[j * NVAR + k] = q[j * NVAR + k] -
                              (G[j * NVAR + k] - G[(j - 1) * NVAR + k]) / dh * (dt / 2.0);

    /* (4) recompute freezing speed and split fluxes at the midpoint */
    for (int j = 1; j + 1 < L; ++j)
        oracle_split_fluxes(h + j * NVAR, d, gamma, p_floor, FRh + j * NVAR,
                            FLh + j * NVAR, cnt);

    /* (5) Eqs. (2ndTVDFluxCorr)-(2ndRFlux) at the midpoint: interfaces
     *     j+1/2 for j = 2 .. n+2 (cells -1 .. n-1).  The left-moving flux is
     *     upwinded from cell j+1 and mirrored about the interface. */
    for (int j = 2; j <= n + 2; ++j) {
        for (int k = 0; k < NVAR; ++k) {
            const double dR1 = (FRh[j * NVAR + k] - FRh[(j - 1) * NVAR + k]) / 2.0;
            const double dR2 = (FRh[(j + 1) * NVAR + k] - FRh[j * NVAR + k]) / 2.0;
            const double R = FRh[j * NVAR + k] + oracle_vanleer(dR1, dR2);

            const double dL1 = (FLh[(j + 1) * NVAR + k] - FLh[(j + 2) * NVAR + k]) / 2.0;
            const double dL2 = (FLh[j * NVAR + k] - FLh[(j + 1) * NVAR + k]) / 2.0;
            const double Lf = FLh[(j + 1) * NVAR + k] + oracle_vanleer(dL1, dL2);

            H[j * NVAR + k] = R - Lf;
        }
    }

    /* (6) Eq. (FullstepValue): full step from u^t, cells 0 .. n-1 */
    for (int i = 0; i < n; ++i) {
        const int j = i + GHOST;
        for (int k = 0; k < NVAR; ++k)
            out[i * NVAR + k] = q[j * NVAR + k] -
                                (H[j * NVAR + k] - H[(j - 1) * NVAR + k]) / dh * dt;
    }

    /* the fluxes through interfaces -1/2 .. n-1/2 (H[j] is interface j+1/2
     * in array index j, so interface i-1/2 is H[i + GHOST - 1]) */
    if (hface)
        for (int i = 0; i <= n; ++i)
            for (int k = 0; k < NVAR; ++k)
                hface[i * NVAR + k] = H[(i + GHOST - 1) * NVAR + k];

    free(FR); free(FL); free(G); free(h); free(FRh); free(FLh); free(H);
}

void oracle_pencil(const double *q, int n, int d, double dt, double dh,
                   double gamma, double p_floor, double *out,
                   oracle_counts *cnt)
{
    oracle_pencil_flux(q, n, d, dt, dh, gamma, p_floor, out, NULL, cnt);
}

/* ---------------------------------------------------------------------- */
/* Block level: dimensional splitting with the region rule                 */
/* ---------------------------------------------------------------------- */

static inline long long cell_index(int m, int x, int y, int z)
{
    return (long long)x + (long long)m * ((long long)y + (long long)m * z);
}

/*
 * One step (one directional triple) on one block.  order = 0 sweeps x, y, z
 * (forward); order = 1 sweeps z, y, x (backward).  in: 5 cubes of (n+6)^3;
 * out: 5 cubes of n^3.
 *
 * flux, if not NULL, receives the block's patch-boundary fluxes (the fluxes
 * across the boundaries of every 8^3 patch of the block, which the closing
 * step of Sec. 3.1 needs for the coarse-fine correction of Sec. 2.1; n must
 * then be a multiple of PATCH).  For each axis d and each face plane f = 0,
 * 8, .., n along d (plane index q = f / 8), the flux through interface f-1/2
 * of the d-pencils with interior transverse coordinates, taken in the sweep
 * along d: flux[((d * NQ + q) * NVAR + k) * n * n + a * n + b], NQ = n/8 + 1,
 * where (a, b) are the two other axes, the higher-numbered one first
 * (x: (z, y); y: (z, x); z: (y, x)) and k the global component.
 */
void oracle_advance_block(const double *in, double *out, int n, int order,
                          double dt, double dh, double gamma, double p_floor,
                          double *flux, oracle_counts *cnt)
{
    const int m = n + 2 * GHOST;
    const long long m3 = (long long)m * m * m;
    double *u = (double *)malloc(sizeof(double) * NVAR * m3);
    memcpy(u, in, sizeof(double) * NVAR * m3);

    const int fwd[3] = {0, 1, 2}, bwd[3] = {2, 1, 0};
    const int *seq = order == 0 ? fwd : bwd;

    double *q = (double *)malloc(sizeof(double) * m * NVAR);
    double *res = (double *)malloc(sizeof(double) * n * NVAR);
    double *hf = (double *)malloc(sizeof(double) * (n + 1) * NVAR);
    const int nq = n / PATCH + 1;

    for (int s = 0; s < 3; ++s) {
        const int d = seq[s];
        /* region rule: an axis swept later in this step keeps its ghosts */
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            int later = 0;
            for (int s2 = s + 1; s2 < 3; ++s2)
                if (seq[s2] == a) later = 1;
            lo[a] = later ? -GHOST : 0;
            hi[a] = later ? n + GHOST : n;
        }
        const int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
        for (int p2 = lo[a2]; p2 < hi[a2]; ++p2) {
            for (int p1 = lo[a1]; p1 < hi[a1]; ++p1) {
                int c[3];
                c[a1] = p1 + GHOST;
                c[a2] = p2 + GHOST;
                for (int j = 0; j < m; ++j) {
                    c[d] = j;
                    const long long idx = cell_index(m, c[0], c[1], c[2]);
                    for (int k = 0; k < NVAR; ++k) q[j * NVAR + k] = u[k * m3 + idx];
                }
                const int interior = p1 >= 0 && p1 < n && p2 >= 0 && p2 < n;
                double *hp = flux && interior ? hf : NULL;
                oracle_pencil_flux(q, n, d, dt, dh, gamma, p_floor, res, hp, cnt);
                for (int i = 0; i < n; ++i) {
                    c[d] = i + GHOST;
                    const long long idx = cell_index(m, c[0], c[1], c[2]);
                    for (int k = 0; k < NVAR; ++k) u[k * m3 + idx] = res[i * NVAR + k];
                }
                if (hp) {
                    /* face coordinates: the higher-numbered transverse axis first */
                    const int a = a1 > a2 ? p1 : p2;
                    const int b = a1 > a2 ? p2 : p1;
                    for (int qq = 0; qq < nq; ++qq)
                        for (int k = 0; k < NVAR; ++k)
                            flux[((long long)(d * nq + qq) * NVAR + k) * n * n + a * n + b] =
                                hf[qq * PATCH * NVAR + k];
                }
            }
        }
    }

    const long long n3 = (long long)n * n * n;
    for (int k = 0; k < NVAR; ++k)
        for (int z = 0; z < n; ++z)
            for (int y = 0; y < n; ++y)
                for (int x = 0; x < n; ++x)
                    out[k * n3 + x + (long long)n * (y + (long long)n * z)] =
                        u[k * m3 + cell_index(m, x + GHOST, y + GHOST, z + GHOST)];

    free(q); free(res); free(hf); free(u);
}

/*
 * One step on a batch of blocks, possibly of different edges, time steps and
 * zone sizes.  Block b reads 5 (edge[b]+6)^3 cubes at in + in_off[b] and
 * writes 5 edge[b]^3 cubes at out + out_off[b] (and, with flux != NULL, its
 * patch-boundary fluxes at flux + flux_off[b]).  Blocks are independent and
 * are spread over OpenMP threads.  Returns the number of threads used.
 */
int oracle_advance_batch(const double *in, double *out, int nblocks,
                         const int *edge, const long long *in_off,
                         const long long *out_off, const double *dt,
                         const double *dh, int order, double gamma,
                         double p_floor, double *flux, const long long *flux_off,
                         long long *n_floored, long long *n_nonphysical)
{
    long long fl = 0, np = 0;
    int nthreads = 1;
#pragma omp parallel reduction(+ : fl, np)
    {
#ifdef _OPENMP
#pragma omp single
        nthreads = omp_get_num_threads();
#endif
        oracle_counts cnt = {0, 0};
#pragma omp for schedule(dynamic, 1)
        for (int b = 0; b < nblocks; ++b)
            oracle_advance_block(in + in_off[b], out + out_off[b], edge[b], order,
                                 dt[b], dh[b], gamma, p_floor,
                                 flux ? flux + flux_off[b] : NULL, &cnt);
        fl += cnt.floored;
        np += cnt.nonphysical;
    }
    if (n_floored) *n_floored = fl;
    if (n_nonphysical) *n_nonphysical = np;
    return nthreads;
}

/* ---------------------------------------------------------------------- */
/* Eq. (CFL): maximum signal speed c_s + max(|v_x|, |v_y|, |v_z|)           */
/* ---------------------------------------------------------------------- */

/*
 * u: five planes of ncells values each, plane k at u + k * plane_stride.
 * The pressure floor rule of the sweeps applies to c_s as well.
 */
double oracle_max_signal_speed(const double *u, long long plane_stride,
                               long long ncells, double gamma, double p_floor)
{
    double smax = 0.0;
    for (long long i = 0; i < ncells; ++i) {
        const double rho = u[i];
        const double vx = u[plane_stride + i] / rho;
        const double vy = u[2 * plane_stride + i] / rho;
        const double vz = u[3 * plane_stride + i] / rho;
        const double e = u[4 * plane_stride + i];
        const double kin = 0.5 * (u[plane_stride + i] * vx + u[2 * plane_stride + i] * vy +
                                  u[3 * plane_stride + i] * vz);
        double P = (gamma - 1.0) * (e - kin);
        if (P < p_floor) P = p_floor;
        const double cs = sqrt(gamma * P / rho);
        double vmax = fabs(vx);
        if (fabs(vy) > vmax) vmax = fabs(vy);
        if (fabs(vz) > vmax) vmax = fabs(vz);
        const double s = cs + vmax;
        if (s > smax) smax = s;
    }
    return smax;
}

/* ---------------------------------------------------------------------- */
/* Conservation sums: Neumaier-compensated sum of x[i] * w                  */
/* ---------------------------------------------------------------------- */

/* Returns sum_i x[i] * w, accumulated with Neumaier's compensation; the
 * final compensation term is written to *comp (the sum already includes it). */
double oracle_compensated_sum(const double *x, long long count, double w,
                              double *comp)
{
    double s = 0.0, c = 0.0;
    for (long long i = 0; i < count; ++i) {
        const double v = x[i] * w;
        const double t = s + v;
        if (fabs(s) >= fabs(v))
            c += (s - t) + v;
        else
            c += (v - t) + s;
        s = t;
    }
    if (comp) *comp = c;
    return s + c;
}
