/* Brute-force FP64 fluence of Eq. 1-3 (test infrastructure only).
 *
 * F(p) = integral over theta of L(p, w(theta)), with no cosine term (Eq. 1),
 * where L is the radiance arriving at p along -w (Eq. 3): the fold of the exact
 * per-cell intervals of Eq. 2-4 over every cell the ray crosses from p to the
 * grid exit, each cell a square of uniform emission and attenuation (Section 5).
 * The angle integral uses M midpoint directions theta_m = 2*pi*(m+1/2)/M.  Cells
 * are walked with the grid traversal of Amanatides and Woo (the method the
 * paper cites for its traced rays), with exact chord lengths.
 *
 * Grid convention: eps and sig are [S][S] row-major, row r, column c; pixel
 * (r, c) is the square [c, c+1) x [r, r+1) in (x, y); p is the pixel centre.
 * Nothing outside the grid emits or attenuates.
 *
 * Shares no code with the HIP library.
 */
#include <math.h>
#include <stddef.h>

static void cell(double eps, double sig, double ell, double *L, double *T) {
    double tau = sig * ell;
    double phi = tau < 1e-5 ? 1.0 - tau / 2.0 + tau * tau / 6.0 : -expm1(-tau) / tau;
    *L = eps * ell * phi;
    *T = exp(-tau);
}

/* Radiance arriving at (px, py) from direction (dx, dy) (the ray runs outwards);
 * *T_exit receives the transmittance from p to the grid's edge. */
static double march(int S, const double *eps, const double *sig,
                    double px, double py, double dx, double dy, double *T_exit) {
    int ix = (int)floor(px), iy = (int)floor(py);
    int stepx = dx > 0 ? 1 : -1, stepy = dy > 0 ? 1 : -1;
    double tdx = dx != 0 ? fabs(1.0 / dx) : INFINITY;
    double tdy = dy != 0 ? fabs(1.0 / dy) : INFINITY;
    double tmx = dx > 0 ? (ix + 1 - px) * tdx : dx < 0 ? (px - ix) * tdx : INFINITY;
    double tmy = dy > 0 ? (iy + 1 - py) * tdy : dy < 0 ? (py - iy) * tdy : INFINITY;
    double t = 0.0, L = 0.0, T = 1.0;
    while (ix >= 0 && ix < S && iy >= 0 && iy < S) {
        double tn = tmx < tmy ? tmx : tmy;
        double ell = tn - t;
        if (ell > 0) {
            double cl, ct;
            size_t id = (size_t)iy * S + ix;
            cell(eps[id], sig[id], ell, &cl, &ct);
            L += T * cl;
            T *= ct;
        }
        t = tn;
        if (tmx < tmy) { ix += stepx; tmx += tdx; }
        else if (tmy < tmx) { iy += stepy; tmy += tdy; }
        else { ix += stepx; iy += stepy; tmx += tdx; tmy += tdy; }
    }
    if (T_exit) *T_exit = T;
    return L;
}

/* Environment radiance seen along the outward direction of angle th (from +x,
 * the column axis, towards +y, the row axis): K samples at angles 2 pi k / K,
 * nearest sample (halfway: the next one counter-clockwise). */
static double env_radiance(const double *env, int K, double th) {
    const double two_pi = 6.283185307179586476925286766559;
    double a = th * K / two_pi;
    long k = (long)floor(a + 0.5);
    k %= K;
    if (k < 0) k += K;
    return env[k];
}

/* Fluence at the centres of rows [r0, r1) x columns [c0, c1); out is
 * [(r1-r0)][(c1-c0)] row-major.  With K > 0 environment samples, light from
 * beyond the grid (vacuum there) adds T_exit times the environment's radiance
 * in the ray's direction.  Returns 0, or -1 on bad arguments. */
int bf_fluence_env(int S, const double *eps, const double *sig, int M,
                   int r0, int r1, int c0, int c1, const double *env, int K, double *out) {
    if (S <= 0 || M <= 0 || r0 < 0 || c0 < 0 || r1 > S || c1 > S || r0 >= r1 || c0 >= c1 ||
        K < 0 || (K > 0 && !env))
        return -1;
    const double two_pi = 6.283185307179586476925286766559;
    int W = c1 - c0, H = r1 - r0;
    long total = (long)W * H;
#pragma omp parallel for schedule(dynamic, 4)
    for (long id = 0; id < total; ++id) {
        int r = r0 + (int)(id / W), c = c0 + (int)(id % W);
        double px = c + 0.5, py = r + 0.5, acc = 0.0;
        for (int m = 0; m < M; ++m) {
            double th = two_pi * (m + 0.5) / M, T_exit = 0.0;
            acc += march(S, eps, sig, px, py, cos(th), sin(th), &T_exit);
            if (K > 0) acc += T_exit * env_radiance(env, K, th);
        }
        out[id] = acc * two_pi / M;
    }
    return 0;
}

int bf_fluence(int S, const double *eps, const double *sig, int M,
               int r0, int r1, int c0, int c1, double *out) {
    return bf_fluence_env(S, eps, sig, M, r0, r1, c0, c1, NULL, 0, out);
}

/* Radiance along a single direction, exposed for unit tests. */
double bf_radiance(int S, const double *eps, const double *sig,
                   double px, double py, double dx, double dy) {
    return march(S, eps, sig, px, py, dx, dy, NULL);
}
