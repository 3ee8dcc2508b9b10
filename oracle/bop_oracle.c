/*
 * CPU oracle for the analytic-BOP energy path — TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the package smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The HIP library never links, calls or includes it,
 * and it includes nothing from the HIP library: the two share no code.
 *
 * Plain, slow, FP64.  Every function follows a passage of Hammerschmidt et al.,
 * "BOPfox program for tight-binding and analytic bond-order potential
 * calculations" (arXiv:1803.07491), cited by section and equation label:
 *
 *   or_neighbours   Sec. II "Initialisation" (pairs within the cutoff, periodic
 *                   images; the paper's ghost-cell picture read as image shifts)
 *   or_build_H      App. A.2.1: bond-frame block Eq. (Hij), bond integrals and
 *                   cutoff Eq. (cutoff), rotation Eq. (Hij_rot), App. D matrices
 *   or_moments      App. B.3: moments Eq. (momDOS) from interference paths built
 *                   iteratively Eq. (xi_rec) and merged Eqs. (xi_invert, xi_merge)
 *   or_recursion    App. B.3: recursion coefficients from moments Eqs. (momtoa,
 *                   momtob) with the c_j^n recursion; App. B.5 Gershgorin band
 *                   edges Eq. (gershogorin) and terminator Eq. (abinf)
 *   or_dos_coeffs   App. B.3 Eq. (sigma_i) and the normalised moments; App. B.4
 *                   chain recursion for higher coefficients Eq. (aexp) and
 *                   Jackson damping Eq. (Jackson)
 *   or_orbital_NU   App. B.2: Chebyshev phase, response functions Eq. (chi),
 *                   N_ia and U_bond,ia; App. A.1 Eq. (TB-Ubond)
 *   or_fermi        Sec. II "DOS and Fermi energy": bisection on the electron count
 *   or_scf_step     App. A.3 Eq. (BOP_LCN) with linear input/output mixing
 *                   (Sec. II "Self-consistency")
 *
 * Readings taken where the paper is silent, garbled or inconsistent are
 * stated next to the code that takes them.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXSP 4
#define OR_NCH 14
/* channel order: sss sps pss sds dss pps ppp pds dps pdp dpp dds ddp ddd */
enum { SSS, SPS, PSS, SDS, DSS, PPS, PPP, PDS, DPS, PDP, DPP, DDS, DDP, DDD };

typedef struct {
    int n_species;
    int n_orb;                       /* 5 (d) or 9 (s, p, d) */
    double r_cut, d_cut;
    double onsite[OR_MAXSP][3];      /* s, p, d level per species */
    int form[OR_MAXSP * OR_MAXSP][OR_NCH];   /* 0 power law, 1 exponential */
    double beta0[OR_MAXSP * OR_MAXSP][OR_NCH];
    double r0[OR_MAXSP * OR_MAXSP][OR_NCH];
    double q[OR_MAXSP * OR_MAXSP][OR_NCH];
} or_model;

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* neighbour list                                                            */
/* ------------------------------------------------------------------------ */

static void inv3(const double *A, double *B)
{
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6])
               + A[2] * (A[3] * A[7] - A[4] * A[6]);
    B[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    B[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
}

/* The pair criterion, evaluated in one fixed order: d = (r_j - r_i) + S.A with
 * S.A = (s1 a1 + s2 a2) + s3 a3 per component, |d|^2 = (dx dx + dy dy) + dz dz,
 * accepted when 0 < |d|^2 < r_cut^2. */
static int pair_vec(const double *pos, const double *A, int i, int j,
                    int s1, int s2, int s3, double rc2, double *d)
{
    for (int k = 0; k < 3; ++k) {
        double sv = ((double)s1 * A[0 + k] + (double)s2 * A[3 + k]) + (double)s3 * A[6 + k];
        d[k] = (pos[3 * j + k] - pos[3 * i + k]) + sv;
    }
    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    return r2 > 0.0 && r2 < rc2;
}

typedef struct { int j, s1, s2, s3; double d[3]; } or_pair;

static int pair_cmp(const void *a, const void *b)
{
    const or_pair *x = (const or_pair *)a, *y = (const or_pair *)b;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    if (x->s1 != y->s1) return x->s1 < y->s1 ? -1 : 1;
    if (x->s2 != y->s2) return x->s2 < y->s2 ? -1 : 1;
    if (x->s3 != y->s3) return x->s3 < y->s3 ? -1 : 1;
    return 0;
}

/* Visit every image S of atom j that can lie within r_cut of atom i: the
 * fractional offset f_j - f_i + S must be smaller than r_cut |g_k| along each
 * reciprocal direction g_k; the range is widened by one on each side. */
static int scan_images(const double *pos, const double *A, const double *f,
                       const double *gn, double rc, int i, int j,
                       or_pair *out, int cap, int cnt)
{
    double rc2 = rc * rc;
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        double df = f[3 * j + k] - f[3 * i + k];
        lo[k] = (int)ceil(-rc * gn[k] - df) - 1;
        hi[k] = (int)floor(rc * gn[k] - df) + 1;
    }
    for (int s1 = lo[0]; s1 <= hi[0]; ++s1)
        for (int s2 = lo[1]; s2 <= hi[1]; ++s2)
            for (int s3 = lo[2]; s3 <= hi[2]; ++s3) {
                double d[3];
                if (!pair_vec(pos, A, i, j, s1, s2, s3, rc2, d)) continue;
                if (cnt < cap) {
                    or_pair *p = &out[cnt];
                    p->j = j; p->s1 = s1; p->s2 = s2; p->s3 = s3;
                    p->d[0] = d[0]; p->d[1] = d[1]; p->d[2] = d[2];
                }
                ++cnt;
            }
    return cnt;
}

/*
 * Periodic neighbour list (Sec. II "Initialisation").  Rows are atoms in
 * input order; each row lists every (j, S) with 0 < |d|^2 < r_cut^2, sorted by
 * (j, s1, s2, s3).  Candidates come from a uniform bin grid over the wrapped
 * fractional coordinates (all bins along an axis with fewer than three bins);
 * `brute` = 1 scans every atom instead.  Returns the total pair count; rows
 * are written only when it fits in `cap`.
 */
long or_neighbours(int n, const double *pos, const double *cell, double rc, int brute,
                   long cap, int *row_ptr, int *nbr_j, int *nbr_shift, double *nbr_d)
{
    double Ainv[9], gn[3];
    inv3(cell, Ainv);
    for (int k = 0; k < 3; ++k)
        gn[k] = sqrt(Ainv[k] * Ainv[k] + Ainv[3 + k] * Ainv[3 + k] + Ainv[6 + k] * Ainv[6 + k]);
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k)
            f[3 * i + k] = pos[3 * i] * Ainv[k] + pos[3 * i + 1] * Ainv[3 + k] + pos[3 * i + 2] * Ainv[6 + k];

    int nb[3];
    for (int k = 0; k < 3; ++k) {
        nb[k] = brute ? 1 : (int)floor(1.0 / (rc * gn[k] * (1.0 + 1e-9)));
        if (nb[k] < 1) nb[k] = 1;
    }
    long nbins = (long)nb[0] * nb[1] * nb[2];
    int *bin_of = (int *)malloc(sizeof(int) * (size_t)n);
    int *bstart = (int *)calloc((size_t)nbins + 1, sizeof(int));
    int *blist = (int *)malloc(sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i) {
        int c[3];
        for (int k = 0; k < 3; ++k) {
            double w = f[3 * i + k] - floor(f[3 * i + k]);
            c[k] = (int)(w * nb[k]);
            if (c[k] >= nb[k]) c[k] = nb[k] - 1;
            if (c[k] < 0) c[k] = 0;
        }
        bin_of[i] = (c[0] * nb[1] + c[1]) * nb[2] + c[2];
        bstart[bin_of[i] + 1]++;
    }
    for (long b = 0; b < nbins; ++b) bstart[b + 1] += bstart[b];
    {
        int *fill = (int *)malloc(sizeof(int) * (size_t)nbins);
        memcpy(fill, bstart, sizeof(int) * (size_t)nbins);
        for (int i = 0; i < n; ++i) blist[fill[bin_of[i]]++] = i;
        free(fill);
    }

    int *cnt = (int *)calloc((size_t)n, sizeof(int));
    int maxrow = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            long tot = 0;
            row_ptr[0] = 0;
            for (int i = 0; i < n; ++i) { tot += cnt[i]; if (cnt[i] > maxrow) maxrow = cnt[i]; }
            if (tot > cap) { free(f); free(bin_of); free(bstart); free(blist); free(cnt); return tot; }
            for (int i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
        }
#pragma omp parallel
        {
            or_pair *buf = (or_pair *)malloc(sizeof(or_pair) * (size_t)(pass ? maxrow + 1 : 1));
#pragma omp for schedule(dynamic, 64)
            for (int i = 0; i < n; ++i) {
                int ci[3] = { bin_of[i] / (nb[1] * nb[2]), (bin_of[i] / nb[2]) % nb[1], bin_of[i] % nb[2] };
                int lo[3], hi[3];
                for (int k = 0; k < 3; ++k) {
                    if (nb[k] >= 3) { lo[k] = ci[k] - 1; hi[k] = ci[k] + 1; }
                    else { lo[k] = 0; hi[k] = nb[k] - 1; }
                }
                int c = 0;
                int cap_i = pass ? cnt[i] : 0;
                for (int x = lo[0]; x <= hi[0]; ++x)
                    for (int y = lo[1]; y <= hi[1]; ++y)
                        for (int z = lo[2]; z <= hi[2]; ++z) {
                            int bx = ((x % nb[0]) + nb[0]) % nb[0];
                            int by = ((y % nb[1]) + nb[1]) % nb[1];
                            int bz = ((z % nb[2]) + nb[2]) % nb[2];
                            int b = (bx * nb[1] + by) * nb[2] + bz;
                            for (int t = bstart[b]; t < bstart[b + 1]; ++t)
                                c = scan_images(pos, cell, f, gn, rc, i, blist[t], buf, cap_i, c);
                        }
                if (!pass) { cnt[i] = c; continue; }
                qsort(buf, (size_t)c, sizeof(or_pair), pair_cmp);
                for (int t = 0; t < c; ++t) {
                    long p = row_ptr[i] + t;
                    nbr_j[p] = buf[t].j;
                    nbr_shift[3 * p] = buf[t].s1;
                    nbr_shift[3 * p + 1] = buf[t].s2;
                    nbr_shift[3 * p + 2] = buf[t].s3;
                    nbr_d[3 * p] = buf[t].d[0];
                    nbr_d[3 * p + 1] = buf[t].d[1];
                    nbr_d[3 * p + 2] = buf[t].d[2];
                }
            }
            free(buf);
        }
    }
    long tot = row_ptr[n];
    free(f); free(bin_of); free(bstart); free(blist); free(cnt);
    return tot;
}

/* ------------------------------------------------------------------------ */
/* Hamiltonian (App. A.2.1 and App. D)                                       */
/* ------------------------------------------------------------------------ */

/* Bond integral beta(r) times the cosine taper Eq. (cutoff) on
 * [r_cut - d_cut, r_cut]; d_cut = 0 means a hard cutoff. */
static double bond_integral(const or_model *m, int pair, int ch, double r)
{
    double b0 = m->beta0[pair][ch];
    if (b0 == 0.0) return 0.0;
    double v;
    if (m->form[pair][ch] == 0) v = b0 * pow(m->r0[pair][ch] / r, m->q[pair][ch]);
    else v = b0 * exp(-m->q[pair][ch] * (r - m->r0[pair][ch]));
    if (m->d_cut > 0.0 && r >= m->r_cut - m->d_cut) {
        double x = (r - (m->r_cut - m->d_cut)) / m->d_cut;
        v *= 0.5 * (cos(M_PI * x) + 1.0);
    }
    return v;
}

/* Rotation matrices of App. D for p (3x3, order p_z, p_x, p_y) and d (5x5,
 * order 3z^2-r^2, zx, yz, x^2-y^2, xy).
 * Reading: theta is the polar angle of the bond from the global z axis and phi
 * its azimuth (App. D's parenthetical "angle to the xy-plane" contradicts both
 * Eq. (Hij_rot) and the matrices themselves); the first index of R_{a,b} names
 * the bond-frame orbital and the second the global one.  The angles enter only
 * through cos/sin, taken from the direction cosines (l, m, n) of the bond:
 * cos(theta) = n, sin(theta) = sqrt(l^2 + m^2), cos(phi) = l / sin(theta),
 * sin(phi) = m / sin(theta), and (cos(phi), sin(phi)) = (1, 0) on the z axis. */
static void rot_p(double ct, double st, double cp, double sp, double R[3][3])
{
    R[0][0] = ct;       R[1][0] = -st;      R[2][0] = 0.0;
    R[0][1] = cp * st;  R[1][1] = cp * ct;  R[2][1] = -sp;
    R[0][2] = sp * st;  R[1][2] = sp * ct;  R[2][2] = cp;
}

static void rot_d(double ct, double st, double cp, double sp, double R[5][5])
{
    const double s3 = sqrt(3.0), s34 = sqrt(0.75);
    double c2t = ct * ct, s2t = st * st, c2p = cp * cp, s2p = sp * sp;
    R[0][0] = c2t - 0.5 * s2t;
    R[1][0] = -s3 * st * ct;
    R[2][0] = 0.0;
    R[3][0] = s34 * s2t;
    R[4][0] = 0.0;
    R[0][1] = s3 * cp * st * ct;
    R[1][1] = cp * (c2t - s2t);
    R[2][1] = -sp * ct;
    R[3][1] = -cp * st * ct;
    R[4][1] = sp * st;
    R[0][2] = s3 * sp * st * ct;
    R[1][2] = sp * (c2t - s2t);
    R[2][2] = cp * ct;
    R[3][2] = -sp * st * ct;
    R[4][2] = -cp * st;
    R[0][3] = (c2p - s2p) * s34 * s2t;
    R[1][3] = (c2p - s2p) * st * ct;
    R[2][3] = -2.0 * sp * cp * st;
    R[3][3] = (c2p - s2p) * (c2t + 0.5 * s2t);
    R[4][3] = -2.0 * sp * cp * ct;
    R[0][4] = s3 * sp * cp * s2t;
    R[1][4] = 2.0 * sp * cp * st * ct;
    R[2][4] = (c2p - s2p) * st;
    R[3][4] = sp * cp * (c2t + 1.0);
    R[4][4] = (c2p - s2p) * ct;
}

/* Exposed for the tests: the App. D matrices for a unit direction u. */
void or_rotation(const double *u, double *Rp9, double *Rd25)
{
    double ct = u[2], st = sqrt(u[0] * u[0] + u[1] * u[1]), cp = 1.0, sp = 0.0;
    if (st > 0.0) { cp = u[0] / st; sp = u[1] / st; }
    double Rp[3][3], Rd[5][5];
    rot_p(ct, st, cp, sp, Rp);
    rot_d(ct, st, cp, sp, Rd);
    memcpy(Rp9, Rp, sizeof Rp);
    memcpy(Rd25, Rd, sizeof Rd);
}

/* Bond-frame block of Eq. (Hij): z' along the bond from atom i to atom j;
 * row = orbital on i, column = orbital on j.  Orbital index: s = 0,
 * p_z p_x p_y = 1..3, d = 4..8 for s,p,d atoms; d-only atoms use d = 0..4. */
static void bond_frame_block(const or_model *m, int pair, double r, double *Hb)
{
    int no = m->n_orb;
    memset(Hb, 0, sizeof(double) * no * no);
    double v[OR_NCH];
    for (int c = 0; c < OR_NCH; ++c) v[c] = bond_integral(m, pair, c, r);
#define HB(a, b) Hb[(a) * no + (b)]
    if (no == 5) {
        HB(0, 0) = v[DDS];
        HB(1, 1) = v[DDP]; HB(2, 2) = v[DDP];
        HB(3, 3) = v[DDD]; HB(4, 4) = v[DDD];
    } else {
        HB(0, 0) = v[SSS]; HB(0, 1) = v[SPS]; HB(0, 4) = v[SDS];
        HB(1, 0) = v[PSS]; HB(1, 1) = v[PPS]; HB(1, 4) = v[PDS];
        HB(2, 2) = v[PPP]; HB(2, 5) = v[PDP];
        HB(3, 3) = v[PPP]; HB(3, 6) = v[PDP];
        HB(4, 0) = v[DSS]; HB(4, 1) = v[DPS]; HB(4, 4) = v[DDS];
        HB(5, 2) = v[DPP]; HB(5, 5) = v[DDP];
        HB(6, 3) = v[DPP]; HB(6, 6) = v[DDP];
        HB(7, 7) = v[DDD]; HB(8, 8) = v[DDD];
    }
#undef HB
}

/*
 * H_on[i][a] = onsite level of atom i's species for orbital a's l, plus the
 * atom's onsite shift (NULL = none).  H_bond[p] = R^T H^(b) R with R the
 * block-diagonal (1, R_p, R_d) rotation, per Eq. (Hij_rot) under the index
 * reading stated at rot_p/rot_d.
 */
void or_build_H(const or_model *m, int n, const int *species, const double *shift,
                const int *row_ptr, const int *nbr_j, const double *nbr_d,
                double *H_on, double *H_bond)
{
    int no = m->n_orb, ns = m->n_species;
    for (int i = 0; i < n; ++i) {
        double sh = shift ? shift[i] : 0.0;
        for (int a = 0; a < no; ++a) {
            int l = (no == 5) ? 2 : (a == 0 ? 0 : (a < 4 ? 1 : 2));
            H_on[(long)i * no + a] = m->onsite[species[i]][l] + sh;
        }
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int j = nbr_j[p];
            const double *d = &nbr_d[3 * (long)p];
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double u[3] = { d[0] / r, d[1] / r, d[2] / r };
            double Rp[9], Rd[25];
            or_rotation(u, Rp, Rd);
            double R[81];
            memset(R, 0, sizeof R);
            if (no == 5) {
                memcpy(R, Rd, sizeof Rd);
            } else {
                R[0] = 1.0;
                for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) R[(1 + a) * 9 + 1 + b] = Rp[a * 3 + b];
                for (int a = 0; a < 5; ++a) for (int b = 0; b < 5; ++b) R[(4 + a) * 9 + 4 + b] = Rd[a * 5 + b];
            }
            double Hb[81], T[81];
            bond_frame_block(m, species[i] * ns + species[j], r, Hb);
            /* T = H^(b) R ; H = R^T T */
            for (int a = 0; a < no; ++a)
                for (int b = 0; b < no; ++b) {
                    double s = 0.0;
                    for (int c = 0; c < no; ++c) s += Hb[a * no + c] * R[c * no + b];
                    T[a * no + b] = s;
                }
            double *H = &H_bond[(long)p * no * no];
            for (int a = 0; a < no; ++a)
                for (int b = 0; b < no; ++b) {
                    double s = 0.0;
                    for (int c = 0; c < no; ++c) s += R[c * no + a] * T[c * no + b];
                    H[a * no + b] = s;
                }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* moments (App. B.3)                                                        */
/* ------------------------------------------------------------------------ */

/*
 * mu[s][a][n] = <i a | H^n | i a> for i = sel[s], n = 0..n_max, where H is the
 * Gamma-point (folded periodic) Hamiltonian: H[i][j] = sum over the list's
 * images S of the block H_ij(S), plus the diagonal onsite levels.
 *
 * Reading: the paper's ghost-cell paths are taken to fold back onto the
 * periodic cell, i.e. paths run on the torus.
 *
 * Interference paths of growing length are built by Eq. (xi_rec):
 * X^k = H X^(k-1), X^0 = the unit columns e_(i a).  The support of X^k is the
 * k-hop neighbourhood of i, found by breadth-first search.  By Eqs. (xi_invert)
 * and (xi_merge) with the split l = floor(n/2):
 *   mu(2k)   = <X^k, X^k>,   mu(2k-1) = <X^(k-1), X^k>,
 *   mu(2K+1) = <X^K, H X^K>  (odd n_max, K = floor(n_max/2)).
 */
int or_moments_radius(int n, int n_orb, int n_max, const int *row_ptr, const int *nbr_j,
                      const double *nbr_d, double r_max, const double *H_on, const double *H_bond,
                      int n_sel, const int *sel, double *mu);

int or_moments(int n, int n_orb, int n_max, const int *row_ptr, const int *nbr_j,
               const double *H_on, const double *H_bond, int n_sel, const int *sel,
               double *mu)
{
    return or_moments_radius(n, n_orb, n_max, row_ptr, nbr_j, NULL, 0.0, H_on, H_bond, n_sel, sel, mu);
}

/*
 * The same with a maximum path radius (Sec. III "Speed-ups" (iii)): when
 * r_max > 0, only interference paths that stay within r_max of their start
 * atom are kept.  The position of a path's end relative to the start atom is
 * the sum of the bond vectors nbr_d along it; a row enters the support only
 * through a bond that ends within r_max, and a bond adds to a row's product
 * only if its target lies within r_max.  (For r_max + r_cut below half the
 * shortest cell height every atom within r_max has one such position.)
 */
int or_moments_radius(int n, int n_orb, int n_max, const int *row_ptr, const int *nbr_j,
                      const double *nbr_d, double r_max, const double *H_on, const double *H_bond,
                      int n_sel, const int *sel, double *mu)
{
    const int trunc = r_max > 0.0 && nbr_d != NULL;
    const double r2max = r_max * r_max;
    int K = n_max / 2, no = n_orb, nb2 = no * no;

#pragma omp parallel
    {
        int *loc = (int *)malloc(sizeof(int) * (size_t)n);
        for (int t = 0; t < n; ++t) loc[t] = -1;
        int cap = 1024;
        int *sup = (int *)malloc(sizeof(int) * cap);
        double *X0 = NULL, *X1 = NULL;
        int xcap = 0;
        int *size = (int *)malloc(sizeof(int) * (K + 2));
        double *rel = (double *)malloc(sizeof(double) * 3 * cap);   /* row position - start position */
#pragma omp for schedule(dynamic, 1)
        for (int s = 0; s < n_sel; ++s) {
            int i = sel[s];
            /* breadth-first layers: size[k] = |support of X^k| */
            int cnt = 0;
            sup[cnt] = i; loc[i] = cnt;
            rel[0] = rel[1] = rel[2] = 0.0;
            ++cnt;
            size[0] = 1;
            for (int k = 1; k <= K; ++k) {
                int begin = (k >= 2) ? size[k - 2] : 0, end = size[k - 1];
                for (int t = begin; t < end; ++t) {
                    int g = sup[t];
                    for (int p = row_ptr[g]; p < row_ptr[g + 1]; ++p) {
                        int j = nbr_j[p];
                        if (loc[j] >= 0) continue;
                        double v[3] = {0.0, 0.0, 0.0};
                        if (trunc) {
                            for (int c = 0; c < 3; ++c) v[c] = rel[3 * t + c] + nbr_d[3 * p + c];
                            if ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2] > r2max) continue;
                        }
                        if (cnt == cap) {
                            cap *= 2;
                            sup = (int *)realloc(sup, sizeof(int) * cap);
                            rel = (double *)realloc(rel, sizeof(double) * 3 * cap);
                        }
                        loc[j] = cnt;
                        for (int c = 0; c < 3; ++c) rel[3 * cnt + c] = v[c];
                        sup[cnt++] = j;
                    }
                }
                size[k] = cnt;
            }
            if (cnt > xcap) {
                xcap = cnt;
                X0 = (double *)realloc(X0, sizeof(double) * (size_t)xcap * nb2);
                X1 = (double *)realloc(X1, sizeof(double) * (size_t)xcap * nb2);
            }
            /* X[r][b][a]: row atom r, its orbital b, start column a */
            memset(X0, 0, sizeof(double) * (size_t)cnt * nb2);
            for (int a = 0; a < no; ++a) X0[a * no + a] = 1.0;
            double *m = &mu[(long)s * no * (n_max + 1)];
            for (int a = 0; a < no; ++a) m[a * (n_max + 1)] = 1.0;
            double *Xp = X0, *Xc = X1;
            int steps = K + (n_max % 2);
            for (int k = 1; k <= steps; ++k) {
                int last = (k > K);              /* H X^K on the rows of X^K only */
                int rows = last ? size[K] : size[k];
                int prev = last ? size[K] : size[k - 1];
                for (int r = 0; r < rows; ++r) {
                    int g = sup[r];
                    double *out = &Xc[(long)r * nb2];
                    for (int t = 0; t < nb2; ++t) out[t] = 0.0;
                    if (r < prev)
                        for (int b = 0; b < no; ++b)
                            for (int a = 0; a < no; ++a)
                                out[b * no + a] = H_on[(long)g * no + b] * Xp[(long)r * nb2 + b * no + a];
                    for (int p = row_ptr[g]; p < row_ptr[g + 1]; ++p) {
                        int lj = loc[nbr_j[p]];
                        if (lj < 0 || lj >= prev) continue;
                        if (trunc) {
                            double v[3];
                            for (int c = 0; c < 3; ++c) v[c] = rel[3 * r + c] + nbr_d[3 * p + c];
                            if ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2] > r2max) continue;
                        }
                        const double *H = &H_bond[(long)p * nb2];
                        const double *x = &Xp[(long)lj * nb2];
                        for (int b = 0; b < no; ++b)
                            for (int c = 0; c < no; ++c) {
                                double h = H[b * no + c];
                                for (int a = 0; a < no; ++a) out[b * no + a] += h * x[c * no + a];
                            }
                    }
                }
                for (int a = 0; a < no; ++a) {
                    double so = 0.0, se = 0.0;
                    for (int r = 0; r < rows; ++r)
                        for (int b = 0; b < no; ++b) {
                            double xc = Xc[(long)r * nb2 + b * no + a];
                            if (r < prev) so += Xp[(long)r * nb2 + b * no + a] * xc;
                            se += xc * xc;
                        }
                    if (last) m[a * (n_max + 1) + 2 * K + 1] = so;
                    else {
                        m[a * (n_max + 1) + 2 * k - 1] = so;
                        m[a * (n_max + 1) + 2 * k] = se;
                    }
                }
                if (!last) { double *tmp = Xp; Xp = Xc; Xc = tmp; }
            }
            for (int t = 0; t < cnt; ++t) loc[sup[t]] = -1;
        }
        free(loc); free(sup); free(X0); free(X1); free(size); free(rel);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* recursion coefficients and band edges (App. B.3, B.5)                     */
/* ------------------------------------------------------------------------ */

#define OR_NMAX 64

int or_n_a(int n_max) { return n_max >= 1 ? (n_max - 1) / 2 + 1 : 0; }
int or_n_b(int n_max) { return n_max / 2; }

/*
 * Per row (one orbital): a_n (n < n_a) and b_n (1 <= n <= n_b, b_0 = 0) from
 * the moments by Eqs. (momtoa, momtob) and the c_j^n recursion.
 *
 * Reading: Eq. (momtob) as printed needs c^n, which itself needs b_n; b_(n+1)
 * is instead taken as the norm of the unnormalised next Lanczos vector,
 * d_j = c_(j-1)^n - a_n c_j^n - b_n c_j^(n-1),  b_(n+1)^2 = sum_jl d_j d_l mu_(j+l),
 * c^(n+1) = d / b_(n+1) — the same recursion solved for b_(n+1).
 * Breakdown (b_(n+1)^2 <= 1e-14 (mu_2 - mu_1^2)): b_(n+1) = 0, the remaining a
 * repeat a_n, the remaining b are 0, flag bit 1 with the level in bits 8+.
 *
 * Band edges: Gershgorin circles Eq. (gershogorin) over the computed rows
 * n = 0..n_a-1, with b_0 = 0 and b_(n_a) included only if it was computed;
 * a_inf = (E_top + E_bot)/2, b_inf = (E_top - E_bot)/4.  bw_mode 1 uses the
 * given global values instead (App. B.5 option (viii)); modes 2-7 are the
 * other estimates of or_band_centre_width.  b_inf below 1e-6 eV is raised to
 * 1e-6 eV (flag bit 8 = value 8).
 */
/*
 * Centre a_inf = A and half-width parameter b_inf = B of the terminator from
 * the computed chain a[0..na-1], b[1..nb] (App. B.5; App. B.1 Eq. weighted).
 *   0  Gershgorin circles, Eq. (gershogorin) (option vii)
 *   1  the given global A = p1, B = p2 (option viii)
 *   2  lowest computed coefficients (option i): A = a_0, B = b_1
 *   3  highest computed coefficients (option ii)
 *   4  averages (option iii): A = mean a_n, B = sqrt(mean b_n^2)
 *   5  average centre, highest width (option iv): A = mean a_n, B = b_top
 *   6  lowest band bottom and highest top (option v, Eq. findeminemax):
 *      A = (max a + min a)/2, B = (max a - min a + 4 max b)/4
 *   7  weighted averages, Eq. (weighted), with beta = p1:
 *      w_m = 1/(beta (M - m) + 1) over m = 0..M for a, 1..M for b
 * Readings: "lowest computed" a is a_0 (the printed a^(1) is the second
 * level of a chain that starts at a^(0), Eq. DOS-G).  The sums and extremes
 * of options i-v and the weighted average run over the levels the chain
 * really computed: up to level L-1 if it broke down at level L (b_L = 0, the
 * later a repeat a_(L-1)); M is the highest such level, separately for a and
 * b.  The weighted average is used as the constant terminator of the tail
 * (Eq. abinf with these values), which also centres and scales the Chebyshev
 * expansion.  Option vi (Beer et al.) and the oscillating terminator need
 * methods the paper only cites and are not provided.
 */
static void or_band_centre_width(int mode, double p1, double p2, const double *ar, const double *br, int na,
                                 int nb, int fl, double *A, double *B)
{
    if (mode == 1) { *A = p1; *B = p2; return; }
    if (mode == 0) {
        double lo = 0.0, hi = 0.0;
        for (int n = 0; n < na; ++n) {
            double bl = (n >= 1 && n <= nb) ? br[n] : 0.0;
            double bh = (n + 1 <= nb) ? br[n + 1] : 0.0;
            double e0 = ar[n] - bl - bh, e1 = ar[n] + bl + bh;
            if (n == 0 || e0 < lo) lo = e0;
            if (n == 0 || e1 > hi) hi = e1;
        }
        *A = 0.5 * (hi + lo);
        *B = 0.25 * (hi - lo);
        return;
    }
    int nav = na, nbv = nb;            /* levels the chain computed */
    if (fl & 1) {
        int L = fl >> 8;
        if (L < nav) nav = L;
        if (L - 1 < nbv) nbv = L - 1;
    }
    double asum = 0.0, amax = 0.0, amin = 0.0, b2sum = 0.0, bmax = 0.0;
    for (int n = 0; n < nav; ++n) {
        asum += ar[n];
        if (n == 0 || ar[n] > amax) amax = ar[n];
        if (n == 0 || ar[n] < amin) amin = ar[n];
    }
    for (int n = 1; n <= nbv; ++n) {
        b2sum += br[n] * br[n];
        if (br[n] > bmax) bmax = br[n];
    }
    double amean = nav > 0 ? asum / nav : 0.0;
    double blow = nbv >= 1 ? br[1] : 0.0, btop = nbv >= 1 ? br[nbv] : 0.0;
    switch (mode) {
    case 2: *A = nav > 0 ? ar[0] : 0.0; *B = blow; break;
    case 3: *A = nav > 0 ? ar[nav - 1] : 0.0; *B = btop; break;
    case 4: *A = amean; *B = nbv > 0 ? sqrt(b2sum / nbv) : 0.0; break;
    case 5: *A = amean; *B = btop; break;
    case 6: *A = 0.5 * (amax + amin); *B = 0.25 * (amax - amin + 4.0 * bmax); break;
    default: {
        double beta = p1, wa = 0.0, sa = 0.0, wb = 0.0, sb = 0.0;
        for (int m = 0; m < nav; ++m) {
            double w = 1.0 / (beta * (double)(nav - 1 - m) + 1.0);
            wa += w; sa += w * ar[m];
        }
        for (int m = 1; m <= nbv; ++m) {
            double w = 1.0 / (beta * (double)(nbv - m) + 1.0);
            wb += w; sb += w * br[m];
        }
        *A = wa > 0.0 ? sa / wa : 0.0;
        *B = wb > 0.0 ? sb / wb : 0.0;
    }
    }
}

void or_recursion(int n_rows, int n_max, const double *mu, int bw_mode,
                  double a_glob, double b_glob, double *a, double *b,
                  double *a_inf, double *b_inf, int *flags)
{
    int na = or_n_a(n_max), nb = or_n_b(n_max);
#pragma omp parallel for schedule(static)
    for (int r = 0; r < n_rows; ++r) {
        double m[2 * OR_NMAX + 2];
        const double *mr = &mu[(long)r * (n_max + 1)];
        for (int t = 0; t <= n_max; ++t) m[t] = mr[t] / mr[0];
        double *ar = &a[(long)r * na], *br = &b[(long)r * (nb + 1)];
        double cprev[OR_NMAX + 2], ccur[OR_NMAX + 2], d[OR_NMAX + 2];
        memset(cprev, 0, sizeof cprev); memset(ccur, 0, sizeof ccur);
        ccur[0] = 1.0;
        br[0] = 0.0;
        int fl = 0, broke = 0;
        double var = (n_max >= 2) ? m[2] - m[1] * m[1] : 0.0;
        for (int n = 0; n < na; ++n) {
            if (broke) { ar[n] = ar[n - 1]; continue; }
            double s = 0.0;
            for (int j = 0; j <= n; ++j)
                for (int l = 0; l <= n; ++l) s += ccur[j] * ccur[l] * m[j + l + 1];
            ar[n] = s;
            if (n + 1 > nb) break;
            for (int j = 0; j <= n + 1; ++j)
                d[j] = (j > 0 ? ccur[j - 1] : 0.0) - ar[n] * ccur[j] - br[n] * cprev[j];
            double b2 = 0.0;
            for (int j = 0; j <= n + 1; ++j)
                for (int l = 0; l <= n + 1; ++l) b2 += d[j] * d[l] * m[j + l];
            if (b2 <= 1e-14 * var) {
                br[n + 1] = 0.0;
                for (int t = n + 2; t <= nb; ++t) br[t] = 0.0;
                fl |= 1 | ((n + 1) << 8);
                broke = 1;
                continue;
            }
            br[n + 1] = sqrt(b2);
            for (int j = 0; j <= n + 1; ++j) { cprev[j] = ccur[j]; ccur[j] = d[j] / br[n + 1]; }
        }
        double ai, bi;
        or_band_centre_width(bw_mode, a_glob, b_glob, ar, br, na, nb, fl, &ai, &bi);
        if (bi < 1e-6) { bi = 1e-6; fl |= 8; }
        a_inf[r] = ai;
        b_inf[r] = bi;
        flags[r] = fl;
    }
}

/* ------------------------------------------------------------------------ */
/* expansion coefficients (App. B.3, B.4)                                    */
/* ------------------------------------------------------------------------ */

/* Jackson kernel Eq. (Jackson) adapted to Chebyshev polynomials of the second
 * kind: g_m = g^J_(m+1) / g^J_1, m = 0..n_exp.
 * Reading: the kernel length is the expansion length, N_J = n_exp (the printed
 * n_max would make g negative beyond n_max while the sum runs to n_exp). */
void or_jackson(int n_exp, double *g)
{
    int NJ = n_exp;
    double w = M_PI / (NJ + 1.0);
    double g1 = ((NJ - 1 + 1) * cos(w * 1) + sin(w * 1) / tan(w)) / (NJ + 1.0);
    for (int m = 0; m <= n_exp; ++m) {
        int mm = m + 1;
        double gj = ((NJ - mm + 1) * cos(w * mm) + sin(w * mm) / tan(w)) / (NJ + 1.0);
        g[m] = gj / g1;
    }
}

/*
 * gsig[r][m] = g_m sigma_m for m = 0..n_exp.
 * For m <= n_max, sigma_m = sum_n p_mn mu^_n (Eq. sigma_i) with the normalised
 * moments mu^_n = (2 b_inf)^-n sum_l C(n,l) (-a_inf)^l mu_(n-l) and p_mn the
 * power coefficients of U_m from p_(m+1)n = 2 p_m(n-1) - p_(m-1)n.
 * For m > n_max, sigma_m = zeta_0^(m) from the chain recursion of App. B.4,
 * zeta_k^(m+1) = 2[a^_k zeta_k^(m) + b^_k zeta_(k-1)^(m) + b^_(k+1) zeta_(k+1)^(m)]
 *                - zeta_k^(m-1),
 * zeta^(0) = e_0, zeta^(-1) = 0, a^_k = (a_k - a_inf)/(2 b_inf),
 * b^_k = b_k / (2 b_inf), and the constant terminator (a^ = 0, b^ = 1/2)
 * beyond the computed levels (Eq. abinf).
 * `sig_chain` (optional, [n_rows][n_max+1]) receives the chain's own values for
 * m <= n_max, which equal the moment route in exact arithmetic.
 * Reading: the first sum of the extended DOS formula in App. B.4 is taken to
 * start at m = 0 (sigma_0 = 1 normalises the DOS).
 * Reading (degenerate band): where the terminator's b_inf sits at its floor
 * (a band of zero width, e.g. an atom without neighbours), the normalised
 * moments divide rounding noise by (2 b_inf)^n and the moment route is
 * meaningless in floating point; such rows take every sigma_m from the chain,
 * which is exact for them (and equal to the moment route in exact arithmetic).
 */
void or_dos_coeffs(int n_rows, int n_max, int n_exp, const double *mu,
                   const double *a, const double *b, const double *a_inf,
                   const double *b_inf, double *gsig, double *sig_chain)
{
    int na = or_n_a(n_max), nb = or_n_b(n_max);
    double *g = (double *)malloc(sizeof(double) * (n_exp + 1));
    or_jackson(n_exp, g);
    /* p_mn for m, n <= n_max */
    int M = n_max + 1;
    double *p = (double *)calloc((size_t)M * M, sizeof(double));
    p[0] = 1.0;
    if (M > 1) p[1 * M + 1] = 2.0;
    for (int m = 1; m + 1 < M; ++m)
        for (int n = 0; n <= m + 1; ++n)
            p[(m + 1) * M + n] = (n >= 1 ? 2.0 * p[m * M + n - 1] : 0.0) - (n <= m - 1 ? p[(m - 1) * M + n] : 0.0);
    /* binomials */
    double *C = (double *)calloc((size_t)M * M, sizeof(double));
    for (int n = 0; n < M; ++n) {
        C[n * M] = 1.0;
        for (int l = 1; l <= n; ++l) C[n * M + l] = C[(n - 1) * M + l - 1] + (l <= n - 1 ? C[(n - 1) * M + l] : 0.0);
    }
#pragma omp parallel
    {
        double *z0 = (double *)malloc(sizeof(double) * (n_exp + 3));
        double *z1 = (double *)malloc(sizeof(double) * (n_exp + 3));
        double *z2 = (double *)malloc(sizeof(double) * (n_exp + 3));
        double *ah = (double *)malloc(sizeof(double) * (n_exp + 3));
        double *bh = (double *)malloc(sizeof(double) * (n_exp + 3));
        double mh[OR_NMAX * 2 + 2], mr[OR_NMAX * 2 + 2];
#pragma omp for schedule(static)
        for (int r = 0; r < n_rows; ++r) {
            double ai = a_inf[r], bi = b_inf[r];
            for (int t = 0; t <= n_max; ++t) mr[t] = mu[(long)r * (n_max + 1) + t] / mu[(long)r * (n_max + 1)];
            for (int n = 0; n <= n_max; ++n) {
                double s = 0.0;
                for (int l = 0; l <= n; ++l) s += C[n * M + l] * pow(-ai, l) * mr[n - l];
                mh[n] = s / pow(2.0 * bi, n);
            }
            double *out = &gsig[(long)r * (n_exp + 1)];
            const int n_mom = bi > 1e-6 ? n_max : 0;
            out[0] = 1.0;
            for (int m = 0; m <= n_mom && m <= n_exp; ++m) {
                double s = 0.0;
                for (int n = 0; n <= m; ++n) s += p[m * M + n] * mh[n];
                out[m] = s;
            }
            /* chain */
            for (int k = 0; k <= n_exp + 2; ++k) {
                ah[k] = (k < na) ? (a[(long)r * na + k] - ai) / (2.0 * bi) : 0.0;
                bh[k] = (k == 0) ? 0.0 : ((k <= nb) ? b[(long)r * (nb + 1) + k] / (2.0 * bi) : 0.5);
                z0[k] = 0.0; z1[k] = 0.0;
            }
            z1[0] = 1.0;                       /* zeta^(0) */
            if (sig_chain) sig_chain[(long)r * (n_max + 1)] = 1.0;
            for (int m = 0; m < n_exp; ++m) {  /* zeta^(m+1) from zeta^(m) = z1, zeta^(m-1) = z0 */
                int top = m + 1 < n_exp + 1 ? m + 1 : n_exp + 1;
                for (int k = 0; k <= top; ++k) {
                    double zm = (k > 0) ? z1[k - 1] : 0.0;
                    double zp = z1[k + 1];
                    z2[k] = 2.0 * (ah[k] * z1[k] + bh[k] * zm + bh[k + 1] * zp) - z0[k];
                }
                for (int k = top + 1; k <= n_exp + 2; ++k) z2[k] = 0.0;
                double *t = z0; z0 = z1; z1 = z2; z2 = t;
                int mm = m + 1;
                if (mm > n_mom) out[mm] = z1[0];
                if (mm <= n_max && sig_chain) sig_chain[(long)r * (n_max + 1) + mm] = z1[0];
            }
            for (int m = 0; m <= n_exp; ++m) out[m] *= g[m];
        }
        free(z0); free(z1); free(z2); free(ah); free(bh);
    }
    free(g); free(p); free(C);
}

/* ------------------------------------------------------------------------ */
/* N, U, DOS per orbital; Fermi level; energies (App. B.2, A.1)             */
/* ------------------------------------------------------------------------ */

/* chi^_m(phi) of App. B.2: chi^_0 = 0, chi^_1 = 1 - phi/pi + sin(2 phi)/(2 pi),
 * chi^_m = [sin((m+1) phi)/(m+1) - sin((m-1) phi)/(m-1)] / pi. */
static double chi_hat(int m, double phi)
{
    if (m == 0) return 0.0;
    if (m == 1) return 1.0 - phi / M_PI + sin(2.0 * phi) / (2.0 * M_PI);
    return (sin((m + 1) * phi) / (m + 1) - sin((m - 1) * phi) / (m - 1)) / M_PI;
}

/*
 * One orbital at energy E: N = sum_m g sigma_m chi^_(m+1)(phi_F) and
 * U = integral up to E of (E' - E_on) n(E') dE', with
 * cos(phi_F) = clamp((E - a_inf)/(2 b_inf), -1, 1).
 * Reading: the phase is eps = +cos(phi) (App. B.2 prints eps = -cos(phi), which
 * contradicts its own Fermi-phase equation and chi^_1); the undefined gamma_0 of
 * the printed U_bond is taken as gamma_0 = (E_on - a_inf)/b_inf, which makes
 * the printed expression equal the onsite form Eq. (TB-Ubond):
 *   U = b_inf sum_m g sigma_m [chi^_(m+2) + chi^_m] + (a_inf - E_on) N.
 * DOS at E: n(E) = (1/(pi b_inf)) sum_m g sigma_m sin((m+1) phi) inside the band.
 */
void or_orbital_NU(int n_exp, const double *gs, double ai, double bi, double e_on,
                   double E, double *N, double *U, double *dos)
{
    double eps = (E - ai) / (2.0 * bi);
    double c = eps < -1.0 ? -1.0 : (eps > 1.0 ? 1.0 : eps);
    double phi = acos(c);
    double sN = 0.0, sU = 0.0, sD = 0.0;
    for (int m = 0; m <= n_exp; ++m) {
        sN += gs[m] * chi_hat(m + 1, phi);
        sU += gs[m] * (chi_hat(m + 2, phi) + chi_hat(m, phi));
        sD += gs[m] * sin((m + 1) * phi);
    }
    if (N) *N = sN;
    if (U) *U = bi * sU + (ai - e_on) * sN;
    if (dos) *dos = (eps > -1.0 && eps < 1.0) ? sD / (M_PI * bi) : 0.0;
}

/* Total electron count (both spins) at E over all orbitals. */
double or_count(int n_rows, int n_exp, const double *gsig, const double *a_inf,
                const double *b_inf, double E)
{
    double tot = 0.0;
#pragma omp parallel for reduction(+ : tot) schedule(static)
    for (int r = 0; r < n_rows; ++r) {
        double N;
        or_orbital_NU(n_exp, &gsig[(long)r * (n_exp + 1)], a_inf[r], b_inf[r], 0.0, E, &N, NULL, NULL);
        tot += N;
    }
    return 2.0 * tot;
}

/*
 * Fermi level by bisection on the total electron count (Sec. II "DOS and Fermi
 * energy").  Reading (bracket and stopping rule are not given): bracket
 * [min(a_inf - 2 b_inf), max(a_inf + 2 b_inf)] over all orbitals; halve while
 * the midpoint differs from both ends, at most 64 times; return the midpoint.
 */
double or_fermi(int n_rows, int n_exp, const double *gsig, const double *a_inf,
                const double *b_inf, double n_elec)
{
    double lo = 0.0, hi = 0.0;
    for (int r = 0; r < n_rows; ++r) {
        double e0 = a_inf[r] - 2.0 * b_inf[r], e1 = a_inf[r] + 2.0 * b_inf[r];
        if (r == 0 || e0 < lo) lo = e0;
        if (r == 0 || e1 > hi) hi = e1;
    }
    for (int it = 0; it < 64; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (or_count(n_rows, n_exp, gsig, a_inf, b_inf, mid) < n_elec) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Per-atom sums over orbitals at E_F, both spins (non-magnetic): N_i, U_i,
 * n_i(E_F); returns U_total = sum_i U_i. */
double or_energy(int n_atoms, int n_orb, int n_exp, const double *gsig,
                 const double *a_inf, const double *b_inf, const double *H_on,
                 double E_F, double *N_atom, double *U_atom, double *dos_atom)
{
    double tot = 0.0;
#pragma omp parallel for reduction(+ : tot) schedule(static)
    for (int i = 0; i < n_atoms; ++i) {
        double sN = 0.0, sU = 0.0, sD = 0.0;
        for (int a = 0; a < n_orb; ++a) {
            long r = (long)i * n_orb + a;
            double N, U, D;
            or_orbital_NU(n_exp, &gsig[r * (n_exp + 1)], a_inf[r], b_inf[r], H_on[r], E_F, &N, &U, &D);
            sN += N; sU += U; sD += D;
        }
        N_atom[i] = 2.0 * sN;
        U_atom[i] = 2.0 * sU;
        dos_atom[i] = 2.0 * sD;
        tot += 2.0 * sU;
    }
    return tot;
}

/*
 * One local-charge-neutrality step (Eq. BOP_LCN, linear mixing).
 * Reading (the update rule and mixing parameter are not given): one onsite
 * shift per atom on all its orbitals; q_i = N_i - N0_i; if max |q_i| < tol the
 * shifts are left as they are (converged); otherwise
 * shift_i += mix q_i / max(n_i(E_F), n_floor) and the mean shift is removed
 * (the pair (shift + c, E_F + c) describes the same state).
 * Returns max |q_i|; *converged = 1 when it is below tol.
 */
double or_scf_step(int n_atoms, const double *N_atom, const double *dos_atom,
                   const double *n0, double mix, double n_floor, double tol,
                   double *shift, double *q, int *converged)
{
    double mq = 0.0;
    for (int i = 0; i < n_atoms; ++i) {
        q[i] = N_atom[i] - n0[i];
        if (fabs(q[i]) > mq) mq = fabs(q[i]);
    }
    *converged = mq < tol;
    if (*converged) return mq;
    double mean = 0.0;
    for (int i = 0; i < n_atoms; ++i) {
        double den = dos_atom[i] > n_floor ? dos_atom[i] : n_floor;
        shift[i] += mix * q[i] / den;
        mean += shift[i];
    }
    mean /= n_atoms;
    for (int i = 0; i < n_atoms; ++i) shift[i] -= mean;
    return mq;
}
