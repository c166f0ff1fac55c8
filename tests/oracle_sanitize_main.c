/*
 * Driver for the sanitizer build of the C oracle (test code only): it runs
 * every entry point of oracle/tvd_oracle.c on small seeded inputs -- a
 * batch of mixed 8^3 and 16^3 ghosted blocks in both sweep orders with and
 * without patch-boundary flux records, single pencils, the signal speed and
 * the compensated sum -- so that an out-of-bounds access, a use of freed
 * memory or undefined behaviour in any of them is reported by
 * -fsanitize=address,undefined.  Exits non-zero on a non-finite result.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_advance_batch(const double *in, double *out, int nblocks, const int *edge,
                         const long long *in_off, const long long *out_off, const double *dt,
                         const double *dh, int order, double gamma, double p_floor,
                         double *flux, const long long *flux_off, long long *n_floored,
                         long long *n_nonphysical);
void oracle_pencil_flux(const double *q, int n, int d, double dt, double dh, double gamma,
                        double p_floor, double *out, double *hface, void *cnt);
double oracle_max_signal_speed(const double *u, long long plane_stride, long long ncells,
                               double gamma, double p_floor);
double oracle_compensated_sum(const double *x, long long count, double w, double *comp);

static unsigned long long state = 88172645463325252ull;
static double uniform01(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0;
}

/* a smooth-ish positive state: rho, m, e with P > 0 */
static void fill_block(double *u, long long m3)
{
    for (long long i = 0; i < m3; ++i) {
        const double rho = 0.5 + uniform01();
        const double vx = uniform01() - 0.5, vy = uniform01() - 0.5, vz = uniform01() - 0.5;
        const double P = 0.2 + uniform01();
        u[i] = rho;
        u[m3 + i] = rho * vx;
        u[2 * m3 + i] = rho * vy;
        u[3 * m3 + i] = rho * vz;
        u[4 * m3 + i] = P / (5.0 / 3.0 - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz);
    }
}

static int all_finite(const double *x, long long n)
{
    for (long long i = 0; i < n; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

int main(void)
{
    const int nb = 5;
    const int edge[5] = {8, 16, 8, 8, 16};
    long long in_off[5], out_off[5], flux_off[5], ni = 0, no = 0, nf = 0;
    double dt[5], dh[5];
    for (int b = 0; b < nb; ++b) {
        const long long n = edge[b], m = n + 6;
        in_off[b] = ni;
        out_off[b] = no;
        flux_off[b] = nf;
        ni += 5 * m * m * m;
        no += 5 * n * n * n;
        nf += 3 * (n / 8 + 1) * 5 * n * n;
        dh[b] = 1.0 / (16.0 * (b + 1));
        dt[b] = 0.05 * dh[b];
    }
    double *in = malloc(sizeof(double) * ni);
    double *out = malloc(sizeof(double) * no);
    double *flux = malloc(sizeof(double) * nf);
    for (int b = 0; b < nb; ++b) {
        const long long m = edge[b] + 6;
        fill_block(in + in_off[b], m * m * m);
    }
    int bad = 0;
    for (int order = 0; order < 2; ++order) {
        for (int rec = 0; rec < 2; ++rec) {
            long long fl = 0, np = 0;
            oracle_advance_batch(in, out, nb, edge, in_off, out_off, dt, dh, order, 5.0 / 3.0,
                                 0.0, rec ? flux : NULL, rec ? flux_off : NULL, &fl, &np);
            bad |= !all_finite(out, no) || (rec && !all_finite(flux, nf)) || np != 0;
        }
    }
    /* pencils of 14 and 22 cells along each axis, with and without records */
    for (int n = 8; n <= 16; n += 8) {
        const int L = n + 6;
        double *q = malloc(sizeof(double) * L * 5);
        double *po = malloc(sizeof(double) * n * 5);
        double *hf = malloc(sizeof(double) * (n + 1) * 5);
        for (int j = 0; j < L; ++j) {
            const double rho = 0.5 + uniform01(), v = uniform01() - 0.5, P = 0.3 + uniform01();
            q[j * 5 + 0] = rho;
            q[j * 5 + 1] = rho * v;
            q[j * 5 + 2] = 0.1 * rho;
            q[j * 5 + 3] = -0.2 * rho;
            q[j * 5 + 4] = 1.5 * P + 0.5 * rho * (v * v + 0.05);
        }
        for (int d = 0; d < 3; ++d) {
            oracle_pencil_flux(q, n, d, 0.01, 0.05, 1.4, 0.0, po, hf, NULL);
            oracle_pencil_flux(q, n, d, 0.01, 0.05, 1.4, 1e-3, po, NULL, NULL);
            bad |= !all_finite(po, n * 5) || !all_finite(hf, (n + 1) * 5);
        }
        free(q);
        free(po);
        free(hf);
    }
    const double s = oracle_max_signal_speed(out, no / 5, no / 5, 5.0 / 3.0, 0.0);
    double comp = 0.0;
    const double sum = oracle_compensated_sum(out, no, 0.5, &comp);
    bad |= !isfinite(s) || !isfinite(sum) || !isfinite(comp);
    free(in);
    free(out);
    free(flux);
    printf("oracle sanitizer driver: %s\n", bad ? "FAILED" : "ok");
    return bad ? 1 : 0;
}
