/* Hard-sphere Monte Carlo moves for the random dense packings of the seeded
 * workloads: the accept/reject loop of workloads.random_dense_packing in C.
 * All random numbers (sweep permutations and trial displacements) are drawn by
 * the caller, so the result is identical to the Python loop. */
#include <math.h>
#include <stdlib.h>

static int bin_of(double x, double w, int nb)
{
    int b = (int)floor(x / w);
    if (b > nb - 1) b = nb - 1;
    if (b < 0) b = 0;
    return b;
}

/* squared distance from point t (in bin tb) to the nearest particle j != i
 * in the 27 surrounding bins; stops early once below `stop` */
static double nearest(int i, const double *t, const int *tb, const double *pos, const int *head,
                      const int *next, int nb, double L, double stop)
{
    double best = 1e300;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                int c = ((((tb[0] + dx) % nb + nb) % nb) * nb + (((tb[1] + dy) % nb + nb) % nb)) * nb
                        + (((tb[2] + dz) % nb + nb) % nb);
                for (int j = head[c]; j >= 0; j = next[j]) {
                    if (j == i) continue;
                    double r2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        double d = t[a] - pos[3 * j + a];
                        d -= L * nearbyint(d / L);
                        r2 += d * d;
                    }
                    if (r2 < best) best = r2;
                    if (best < stop) return best;
                }
            }
    return best;
}

/* pos [n][3] in/out; perm [sweeps][n]; disp [sweeps][n][3] in [-step, step] */
void rdp_sweeps(int n, double L, double dmin, int nb, int sweeps, const long *perm, const double *disp,
                double *pos)
{
    const double w = L / nb;
    int *head = (int *)malloc(sizeof(int) * nb * nb * nb), *next = (int *)malloc(sizeof(int) * n);
    int *prev = (int *)malloc(sizeof(int) * n), *bin = (int *)malloc(sizeof(int) * n);
    for (int c = 0; c < nb * nb * nb; ++c) head[c] = -1;
    /* per-bin doubly linked lists; insertion order matches the Python lists */
    int *tail = (int *)malloc(sizeof(int) * nb * nb * nb);
    for (int c = 0; c < nb * nb * nb; ++c) tail[c] = -1;
    for (int i = 0; i < n; ++i) {
        int c = (bin_of(pos[3 * i], w, nb) * nb + bin_of(pos[3 * i + 1], w, nb)) * nb + bin_of(pos[3 * i + 2], w, nb);
        bin[i] = c; next[i] = -1; prev[i] = tail[c];
        if (tail[c] >= 0) next[tail[c]] = i; else head[c] = i;
        tail[c] = i;
    }
    for (int s = 0; s < sweeps; ++s) {
        for (int q = 0; q < n; ++q) {
            const int i = (int)perm[(long)s * n + q];
            const double *dd = disp + ((long)s * n + q) * 3;
            double t[3];
            for (int a = 0; a < 3; ++a) {
                t[a] = fmod(pos[3 * i + a] + dd[a], L);
                if (t[a] < 0) t[a] += L;
            }
            int tb[3] = {bin_of(t[0], w, nb), bin_of(t[1], w, nb), bin_of(t[2], w, nb)};
            /* accept if the trial keeps dmin from everyone, or (start-up
             * overlaps) if it strictly increases i's nearest distance */
            const double mt = nearest(i, t, tb, pos, head, next, nb, L, dmin * dmin);
            int ok = mt >= dmin * dmin;
            if (!ok) {
                const int cb[3] = {bin[i] / (nb * nb), (bin[i] / nb) % nb, bin[i] % nb};
                const double mc = nearest(i, pos + 3 * i, cb, pos, head, next, nb, L, -1.0);
                ok = nearest(i, t, tb, pos, head, next, nb, L, -1.0) > mc;
            }
            if (!ok) continue;
            const int ob = bin[i], nbn = (tb[0] * nb + tb[1]) * nb + tb[2];
            /* unlink from the old bin, append to the new one */
            if (prev[i] >= 0) next[prev[i]] = next[i]; else head[ob] = next[i];
            if (next[i] >= 0) prev[next[i]] = prev[i]; else tail[ob] = prev[i];
            next[i] = -1; prev[i] = tail[nbn];
            if (tail[nbn] >= 0) next[tail[nbn]] = i; else head[nbn] = i;
            tail[nbn] = i;
            bin[i] = nbn;
            for (int a = 0; a < 3; ++a) pos[3 * i + a] = t[a];
        }
    }
    free(head); free(next); free(prev); free(bin); free(tail);
}
