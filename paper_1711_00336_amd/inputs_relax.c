/*
 * Geometric overlap removal for the seeded sphere packings of inputs.py.
 * Not part of the method: overlapping pairs are pushed apart along their
 * centre line by half the overlap each (Gauss-Seidel sweeps over a cell
 * list), walls clamp centres to [r, L - r], periodic axes wrap.
 *
 * Cells are visited in 27 colour classes (cell coordinates mod 3); cells of
 * one class have disjoint 3x3x3 neighbourhoods, so a class is processed in
 * parallel (OpenMP) and the result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double wrapd(double x, double L)
{
    if (x >= L) x -= L * floor(x / L);
    else if (x < 0.0) x -= L * floor(x / L);
    if (x >= L) x = 0.0;
    return x;
}

/* lpos, lr: positions and radii in cell order (slot t holds particle
 * order[t]); pairs are still taken in ascending particle index, so the
 * sweep is the same as one over the particle-indexed arrays, only with the
 * neighbours of a cell stored next to each other. The neighbour cells are
 * visited z, y, then x; three x-neighbours that do not wrap are one
 * contiguous slot range. */
static void relax_cell(int64_t c, int cx, int cy, int cz, const int nb[3], const int64_t *start,
                       const int64_t *order, double *lpos, const double *lr, const double *box, const int32_t *per,
                       double tol, double *maxov_out)
{
    double maxov = *maxov_out;
    const double hbox[3] = {0.5 * box[0], 0.5 * box[1], 0.5 * box[2]};
    /* slot ranges of the neighbour cells, in visiting order */
    int64_t rlo[27], rhi[27];
    int nr = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
            int qy = cy + dy, qz = cz + dz;
            if (qy < 0 || qy >= nb[1]) {
                if (!per[1]) continue;
                qy = (qy + nb[1]) % nb[1];
            }
            if (qz < 0 || qz >= nb[2]) {
                if (!per[2]) continue;
                qz = (qz + nb[2]) % nb[2];
            }
            /* with fewer than 3 cells on an axis a neighbour cell repeats;
             * visit each distinct cell once */
            if ((nb[1] == 1 && dy != 0) || (nb[1] == 2 && dy == 1)) continue;
            if ((nb[2] == 1 && dz != 0) || (nb[2] == 2 && dz == 1)) continue;
            const int64_t row = (int64_t)nb[0] * (qy + (int64_t)nb[1] * qz);
            if (cx >= 1 && cx + 1 < nb[0]) {
                rlo[nr] = start[row + cx - 1];
                rhi[nr] = start[row + cx + 2];
                ++nr;
                continue;
            }
            for (int dx = -1; dx <= 1; ++dx) {
                int qx = cx + dx;
                if (qx < 0 || qx >= nb[0]) {
                    if (!per[0]) continue;
                    qx = (qx + nb[0]) % nb[0];
                }
                if ((nb[0] == 1 && dx != 0) || (nb[0] == 2 && dx == 1)) continue;
                rlo[nr] = start[row + qx];
                rhi[nr] = start[row + qx + 1];
                ++nr;
            }
        }
    for (int64_t t = start[c]; t < start[c + 1]; ++t) {
        const int64_t i = order[t];
        for (int k = 0; k < nr; ++k)
            for (int64_t u = rlo[k]; u < rhi[k]; ++u) {
                const int64_t j = order[u];
                if (j <= i) continue;
                double d[3], d2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    d[a] = lpos[3 * u + a] - lpos[3 * t + a];
                    /* minimum image; nearbyint(d/L) is 0 for |d| <= L/2 */
                    if (per[a] && fabs(d[a]) > hbox[a]) d[a] -= box[a] * nearbyint(d[a] / box[a]);
                    d2 += d[a] * d[a];
                }
                const double s = lr[t] + lr[u];
                if (d2 >= s * s) continue;
                const double dist = sqrt(d2);
                const double ov = s - dist;
                if (ov > maxov) maxov = ov;
                const double push = 0.5 * ov + 0.5 * tol;
                double nrm[3];
                for (int a = 0; a < 3; ++a) nrm[a] = dist > 1e-12 ? d[a] / dist : (a == 0 ? 1.0 : 0.0);
                for (int a = 0; a < 3; ++a) {
                    lpos[3 * t + a] -= push * nrm[a];
                    lpos[3 * u + a] += push * nrm[a];
                }
            }
    }
    *maxov_out = maxov;
}

/* returns the number of sweeps used, or -1 if max_sweeps was reached;
 * nthreads > 0 sets the OpenMP thread count (the result does not depend on
 * it), 0 keeps the default */
int lbdem_inputs_relax(int64_t n, double *pos, const double *r, const double *box, const int32_t *per,
                       double tol, int32_t max_sweeps, int32_t nthreads)
{
    if (n <= 1) return 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    double rmax = 0.0;
    for (int64_t i = 0; i < n; ++i) rmax = fmax(rmax, r[i]);
    int nb[3];
    double cs[3];
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        nb[a] = (int)floor(box[a] / (2.0 * rmax));
        if (nb[a] < 1) nb[a] = 1;
        /* periodic axes: a multiple of 3 cells, so colour classes stay apart
         * across the wrap (cells only grow) */
        if (per[a] && nb[a] >= 3) nb[a] -= nb[a] % 3;
        cs[a] = box[a] / nb[a];
        ncell *= nb[a];
    }
    const int serial = nb[0] < 3 || nb[1] < 3 || nb[2] < 3;
    int64_t *start = malloc(sizeof(int64_t) * (size_t)(ncell + 1));
    int64_t *cnt = malloc(sizeof(int64_t) * (size_t)ncell);
    int64_t *order = malloc(sizeof(int64_t) * (size_t)n);
    int64_t *cell = malloc(sizeof(int64_t) * (size_t)n);
    double *lpos = malloc(sizeof(double) * 3 * (size_t)n);
    double *lr = malloc(sizeof(double) * (size_t)n);
    int result = -1;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        memset(cnt, 0, sizeof(int64_t) * (size_t)ncell);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int b[3];
            for (int a = 0; a < 3; ++a) {
                b[a] = (int)floor(pos[3 * i + a] / cs[a]);
                if (b[a] < 0) b[a] = 0;
                if (b[a] >= nb[a]) b[a] = nb[a] - 1;
            }
            cell[i] = b[0] + (int64_t)nb[0] * (b[1] + (int64_t)nb[1] * b[2]);
        }
        for (int64_t i = 0; i < n; ++i) cnt[cell[i]]++;
        start[0] = 0;
        for (int64_t c = 0; c < ncell; ++c) start[c + 1] = start[c] + cnt[c];
        memset(cnt, 0, sizeof(int64_t) * (size_t)ncell);
        for (int64_t i = 0; i < n; ++i) order[start[cell[i]] + cnt[cell[i]]++] = i;
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < n; ++t) {
            const int64_t i = order[t];
            for (int a = 0; a < 3; ++a) lpos[3 * t + a] = pos[3 * i + a];
            lr[t] = r[i];
        }
        double maxov = 0.0;
        for (int color = 0; color < 27; ++color) {
            const int ox = color % 3, oy = (color / 3) % 3, oz = color / 9;
            const int mx = (nb[0] - ox + 2) / 3, my = (nb[1] - oy + 2) / 3, mz = (nb[2] - oz + 2) / 3;
            const int64_t mcells = (int64_t)mx * my * mz;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : maxov) if (!serial)
            for (int64_t m = 0; m < mcells; ++m) {
                const int cx = ox + 3 * (int)(m % mx), cy = oy + 3 * (int)((m / mx) % my),
                          cz = oz + 3 * (int)(m / ((int64_t)mx * my));
                const int64_t c = cx + (int64_t)nb[0] * (cy + (int64_t)nb[1] * cz);
                relax_cell(c, cx, cy, cz, nb, start, order, lpos, lr, box, per, tol, &maxov);
            }
        }
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < n; ++t) {
            const int64_t i = order[t];
            for (int a = 0; a < 3; ++a) {
                double x = lpos[3 * t + a];
                if (per[a]) x = wrapd(x, box[a]);
                else {
                    if (x < r[i]) x = r[i];
                    if (x > box[a] - r[i]) x = box[a] - r[i];
                }
                pos[3 * i + a] = x;
            }
        }
        if (maxov < tol) {
            result = sweep + 1;
            break;
        }
    }
    free(lpos);
    free(lr);
    free(start);
    free(cnt);
    free(order);
    free(cell);
    return result;
}
