// FP64 tail of the energy path (App. B of arXiv:1803.07491):
//  * recursion coefficients from moments (App. B.3, Eqs. momtoa, momtob and the
//    c_j^n recursion) with the Gershgorin terminator (App. B.5, Eq. gershogorin);
//  * Chebyshev expansion coefficients sigma_m (Eq. sigma_i), extended beyond
//    n_max by the chain recursion of App. B.4 with the constant terminator, and
//    Jackson damping (Eq. Jackson);
//  * electron counts, bond energies and DOS at E (App. B.2), the Fermi level
//    by bisection (Sec. II), four halvings per pass over the coefficients,
//    per-atom sums (App. A.1 Eq. TB-Ubond).
//
// The chain recursion is evaluated on the computed levels 0..L-1 plus one
// level L: beyond the computed coefficients the terminated chain is free
// (a^ = 0, b^ = 1/2), and a free semi-infinite chain started from rest only
// passes its input down with a delay of one step, so level L obeys
// zeta_L^(m+1) = 2 b^_L zeta_(L-1)^(m) exactly and the levels below it see the
// same values as with the infinite tail.  Each row's chain then fits in
// registers.
//
// Expansion coefficients are stored m-major ([n_exp+1][rows]) so that the
// per-orbital sums read coalesced columns.  Global sums (electron count,
// bracket, total energy) use per-block partials reduced in a fixed order by a
// one-block launch that follows, so results are deterministic and no block
// needs a device-scope fence (which would write back L2).
#include "bop_internal.h"

#include <cmath>
#include <mutex>

namespace bop {
namespace {

constexpr int MAX_NMAX = 40;
constexpr int DT = 256;        // threads per block in this file

__device__ inline int n_a_of(int n_max) { return n_max >= 1 ? (n_max - 1) / 2 + 1 : 0; }
__device__ inline int n_b_of(int n_max) { return n_max / 2; }

// ---------------------------------------------------------------------------
// recursion coefficients and band edges
// ---------------------------------------------------------------------------
// Centre and width of the terminator from a row's stored chain a[0..na-1],
// b[1..nb] for the estimates of App. B.5 other than Gershgorin and the global
// values: (i) lowest, (ii) highest computed levels, (iii) averages, (iv)
// average centre with the highest width, (v) extreme a with the largest b
// (Eq. findeminemax), and the weighted averages of Eq. (weighted) with
// w_m = 1 / (beta (M - m) + 1).  Only the levels the chain computed count: up
// to level L - 1 when it broke down at level L (flag level L).
__device__ inline void band_estimate(int mode, double beta, const double *ar, const double *br, int na, int nb,
                                     int fl, double &A, double &B)
{
    int nav = na, nbv = nb;
    if (fl & BOP_FLAG_BREAKDOWN) {
        const int L = fl >> 8;
        nav = min(nav, L);
        nbv = min(nbv, L - 1);
    }
    double asum = 0.0, amax = 0.0, amin = 0.0, b2sum = 0.0, bmax = 0.0;
    for (int n = 0; n < nav; ++n) {
        const double v = ar[n];
        asum += v;
        amax = n == 0 ? v : fmax(amax, v);
        amin = n == 0 ? v : fmin(amin, v);
    }
    for (int n = 1; n <= nbv; ++n) {
        const double v = br[n];
        b2sum += v * v;
        bmax = fmax(bmax, v);
    }
    const double amean = nav > 0 ? asum / nav : 0.0;
    const double blow = nbv >= 1 ? br[1] : 0.0, btop = nbv >= 1 ? br[nbv] : 0.0;
    switch (mode) {
    case BOP_BW_LOWEST: A = nav > 0 ? ar[0] : 0.0; B = blow; break;
    case BOP_BW_HIGHEST: A = nav > 0 ? ar[nav - 1] : 0.0; B = btop; break;
    case BOP_BW_AVERAGE: A = amean; B = nbv > 0 ? sqrt(b2sum / nbv) : 0.0; break;
    case BOP_BW_AVERAGE_HIGHEST: A = amean; B = btop; break;
    case BOP_BW_MINMAX: A = 0.5 * (amax + amin); B = 0.25 * (amax - amin + 4.0 * bmax); break;
    default: {
        double wa = 0.0, sa = 0.0, wb = 0.0, sb = 0.0;
        for (int m = 0; m < nav; ++m) {
            const double w = 1.0 / (beta * (double)(nav - 1 - m) + 1.0);
            wa += w;
            sa += w * ar[m];
        }
        for (int m = 1; m <= nbv; ++m) {
            const double w = 1.0 / (beta * (double)(nbv - m) + 1.0);
            wb += w;
            sb += w * br[m];
        }
        A = wa > 0.0 ? sa / wa : 0.0;
        B = wb > 0.0 ? sb / wb : 0.0;
    }
    }
}
__global__ void __launch_bounds__(DT)
k_recursion(int n_rows, int n_max, const double *__restrict__ mu, int bw_mode, double a_glob,
            double b_glob, double *__restrict__ a, double *__restrict__ b, double *__restrict__ a_inf,
            double *__restrict__ b_inf, int *__restrict__ flags)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int na = n_a_of(n_max), nb = n_b_of(n_max);
    double *ar = a + (long)r * na, *br = b + (long)r * (nb + 1);
    int fl = 0;
    if (!mu) {
        // a, b given (Lanczos form); keep its breakdown and non-finite flags
        fl = flags[r];
        goto terminator;
    }
    {
    double m[MAX_NMAX + 1];
    const double *mr = mu + (long)r * (n_max + 1);
    const double m0 = mr[0];
    for (int t = 0; t <= n_max; ++t) {
        m[t] = mr[t] / m0;
        if (!isfinite(m[t])) fl |= BOP_FLAG_NONFINITE;
    }
    double cp[MAX_NMAX / 2 + 3], cc[MAX_NMAX / 2 + 3], d[MAX_NMAX / 2 + 3];
    for (int j = 0; j < MAX_NMAX / 2 + 3; ++j) { cp[j] = 0.0; cc[j] = 0.0; }
    cc[0] = 1.0;
    br[0] = 0.0;
    double bn = 0.0;                   // b_n of the current level
    const double var = (n_max >= 2) ? m[2] - m[1] * m[1] : 0.0;
    bool broke = false;
    for (int n = 0; n < na; ++n) {
        if (broke) { ar[n] = ar[n - 1]; continue; }
        double s = 0.0;
        for (int j = 0; j <= n; ++j)
            for (int l = 0; l <= n; ++l) s += cc[j] * cc[l] * m[j + l + 1];
        ar[n] = s;
        if (n + 1 > nb) break;
        for (int j = 0; j <= n + 1; ++j) d[j] = (j > 0 ? cc[j - 1] : 0.0) - s * cc[j] - bn * cp[j];
        double b2 = 0.0;
        for (int j = 0; j <= n + 1; ++j)
            for (int l = 0; l <= n + 1; ++l) b2 += d[j] * d[l] * m[j + l];
        if (!(b2 > 1e-14 * var)) {
            for (int t = n + 1; t <= nb; ++t) br[t] = 0.0;
            fl |= BOP_FLAG_BREAKDOWN | ((n + 1) << 8);
            broke = true;
            continue;
        }
        double bb = sqrt(b2);
        br[n + 1] = bb;
        for (int j = 0; j <= n + 1; ++j) { cp[j] = cc[j]; cc[j] = d[j] / bb; }
        bn = bb;
    }
    }
terminator:
    double ai, bi;
    if (bw_mode == BOP_BW_GLOBAL) { ai = a_glob; bi = b_glob; }
    else if (bw_mode != BOP_BW_GERSHGORIN) band_estimate(bw_mode, a_glob, ar, br, na, nb, fl, ai, bi);
    else {
        double lo = 0.0, hi = 0.0;
        for (int n = 0; n < na; ++n) {
            double bl = (n >= 1 && n <= nb) ? br[n] : 0.0;
            double bh = (n + 1 <= nb) ? br[n + 1] : 0.0;
            double e0 = ar[n] - bl - bh, e1 = ar[n] + bl + bh;
            if (n == 0 || e0 < lo) lo = e0;
            if (n == 0 || e1 > hi) hi = e1;
        }
        ai = 0.5 * (hi + lo);
        bi = 0.25 * (hi - lo);
    }
    if (!(bi >= 1e-6)) { bi = 1e-6; fl |= BOP_FLAG_NARROW; }
    a_inf[r] = ai;
    b_inf[r] = bi;
    flags[r] = fl;
}

// The same recursion with its arrays in registers, for moments up to NM: the
// loops over the levels and orbital indices are unrolled with compile-time
// bounds, so no array needs indexing at run time.  The additions are the
// generic kernel's, in the same order.
template <int NM>
__global__ void __launch_bounds__(DT)
k_recursion_reg(int n_rows, int n_max, const double *__restrict__ mu, int bw_mode, double a_glob,
                double b_glob, double *__restrict__ a, double *__restrict__ b, double *__restrict__ a_inf,
                double *__restrict__ b_inf, int *__restrict__ flags)
{
    constexpr int NA = (NM - 1) / 2 + 1;       // levels of a
    constexpr int NB = NM / 2;                  // levels of b
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int na = n_a_of(n_max), nb = n_b_of(n_max);
    double *ar = a + (long)r * na, *br = b + (long)r * (nb + 1);
    int fl = 0;
    double m[NM + 1];
    const double *mr = mu + (long)r * (n_max + 1);
    const double m0 = mr[0];
#pragma unroll
    for (int t = 0; t <= NM; ++t) {
        m[t] = (t <= n_max) ? mr[t] / m0 : 0.0;
        if (t <= n_max && !isfinite(m[t])) fl |= BOP_FLAG_NONFINITE;
    }
    double av[NA], bv[NB + 2];
    double cp[NB + 2], cc[NB + 2], d[NB + 2];
#pragma unroll
    for (int j = 0; j < NB + 2; ++j) { cp[j] = 0.0; cc[j] = 0.0; d[j] = 0.0; bv[j] = 0.0; }
    cc[0] = 1.0;
    double bn = 0.0;
    const double var = (n_max >= 2) ? m[2] - m[1] * m[1] : 0.0;
    bool broke = false, done = false;
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        av[n] = 0.0;
        if (n >= na || done) continue;
        if (broke) { av[n] = av[n > 0 ? n - 1 : 0]; continue; }
        double s = 0.0;
#pragma unroll
        for (int j = 0; j <= n; ++j)
#pragma unroll
            for (int l = 0; l <= n; ++l) s += cc[j] * cc[l] * m[j + l + 1];
        av[n] = s;
        if (n + 1 > nb) { done = true; continue; }
#pragma unroll
        for (int j = 0; j <= n + 1; ++j) d[j] = (j > 0 ? cc[j - 1] : 0.0) - s * cc[j] - bn * cp[j];
        double b2 = 0.0;
#pragma unroll
        for (int j = 0; j <= n + 1; ++j)
#pragma unroll
            for (int l = 0; l <= n + 1; ++l) b2 += d[j] * d[l] * m[j + l];
        if (!(b2 > 1e-14 * var)) {
            fl |= BOP_FLAG_BREAKDOWN | ((n + 1) << 8);
            broke = true;
            continue;
        }
        const double bb = sqrt(b2);
        bv[n + 1] = bb;
#pragma unroll
        for (int j = 0; j <= n + 1; ++j) { cp[j] = cc[j]; cc[j] = d[j] / bb; }
        bn = bb;
    }
#pragma unroll
    for (int n = 0; n < NA; ++n)
        if (n < na) ar[n] = av[n];
#pragma unroll
    for (int n = 0; n <= NB; ++n)
        if (n <= nb) br[n] = bv[n];
    double ai, bi;
    if (bw_mode == 1) { ai = a_glob; bi = b_glob; }
    else {
        double lo = 0.0, hi = 0.0;
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            if (n >= na) continue;
            const double bl = (n >= 1 && n <= nb) ? bv[n] : 0.0;
            const double bh = (n + 1 <= nb) ? bv[n + 1] : 0.0;
            const double e0 = av[n] - bl - bh, e1 = av[n] + bl + bh;
            if (n == 0 || e0 < lo) lo = e0;
            if (n == 0 || e1 > hi) hi = e1;
        }
        ai = 0.5 * (hi + lo);
        bi = 0.25 * (hi - lo);
    }
    if (!(bi >= 1e-6)) { bi = 1e-6; fl |= BOP_FLAG_NARROW; }
    a_inf[r] = ai;
    b_inf[r] = bi;
    flags[r] = fl;
}

// ---------------------------------------------------------------------------
// expansion coefficients g_m sigma_m, m-major
// ---------------------------------------------------------------------------
template <int LM>
__global__ void __launch_bounds__(DT)
k_dos_coeffs(int n_rows, int n_max, int n_exp, const double *__restrict__ mu,
             const double *__restrict__ a, const double *__restrict__ b,
             const double *__restrict__ a_inf, const double *__restrict__ b_inf,
             double *__restrict__ gs, int *__restrict__ flags)
{
    __shared__ double s_p[(MAX_NMAX + 1) * (MAX_NMAX + 1)];   // p_mn
    __shared__ double s_c[(MAX_NMAX + 1) * (MAX_NMAX + 1)];   // binomials
    __shared__ double s_g[1025];                              // Jackson g_m
    const int M = n_max + 1;
    if (threadIdx.x == 0) {
        for (int t = 0; t < M * M; ++t) { s_p[t] = 0.0; s_c[t] = 0.0; }
        s_p[0] = 1.0;
        if (M > 1) s_p[M + 1] = 2.0;
        for (int m = 1; m + 1 < M; ++m)
            for (int n = 0; n <= m + 1; ++n)
                s_p[(m + 1) * M + n] = (n >= 1 ? 2.0 * s_p[m * M + n - 1] : 0.0) - (n <= m - 1 ? s_p[(m - 1) * M + n] : 0.0);
        for (int n = 0; n < M; ++n) {
            s_c[n * M] = 1.0;
            for (int l = 1; l <= n; ++l) s_c[n * M + l] = s_c[(n - 1) * M + l - 1] + (l <= n - 1 ? s_c[(n - 1) * M + l] : 0.0);
        }
    }
    {
        // Jackson kernel of length n_exp adapted to U polynomials: g_m = g^J_(m+1)/g^J_1
        const double w = M_PI / (n_exp + 1.0);
        const double cotw = cos(w) / sin(w);
        const double g1 = ((double)n_exp * cos(w) + sin(w) * cotw) / (n_exp + 1.0);
        for (int m = threadIdx.x; m <= n_exp; m += blockDim.x) {
            int mm = m + 1;
            double gj = ((double)(n_exp - mm + 1) * cos(w * mm) + sin(w * mm) * cotw) / (n_exp + 1.0);
            s_g[m] = gj / g1;
        }
    }
    __syncthreads();
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int na = n_a_of(n_max), nb = n_b_of(n_max);
    const double ai = a_inf[r], bi = b_inf[r];
    // Every sigma_m comes from the chain without moments (Lanczos form) and for
    // a band of zero width (b_inf at its floor), where the normalised moments
    // would divide rounding noise by (2 b_inf)^n.
    const int n_mom = (mu && bi > 1e-6) ? n_max : 0;
    double big = 0.0;          // |g sigma| of a proper DOS stays below m + 1
    if (n_mom == 0) {
        gs[r] = s_g[0];
    } else {
    const double *mr = mu + (long)r * M;
    // normalised moments mu^_n
    double mh[MAX_NMAX + 1];
    const double m0 = mr[0];
    for (int n = 0; n < M; ++n) {
        double s = 0.0, pa = 1.0;           // pa = (-a_inf)^l
        for (int l = 0; l <= n; ++l) {
            s += s_c[n * M + l] * pa * (mr[n - l] / m0);
            pa *= -ai;
        }
        mh[n] = s / pow(2.0 * bi, (double)n);
    }
    for (int m = 0; m < M && m <= n_exp; ++m) {
        double s = 0.0;
        for (int n = 0; n <= m; ++n) s += s_p[m * M + n] * mh[n];
        gs[(long)m * n_rows + r] = s_g[m] * s;
        big = fmax(big, fabs(s_g[m] * s));
    }
    }
    if (n_exp <= n_mom) {
        if (!(big <= 1e4)) flags[r] |= BOP_FLAG_DIVERGENT;
        return;
    }
    // chain on levels 0..L with the delay level L
    const int L = na > nb ? na : nb;
    double ah[LM + 1], bh[LM + 2], z0[LM + 1], z1[LM + 1];
#pragma unroll
    for (int k = 0; k <= LM; ++k) {
        ah[k] = (k < na) ? (a[(long)r * na + k] - ai) / (2.0 * bi) : 0.0;
        z0[k] = 0.0;
        z1[k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k <= LM + 1; ++k)
        bh[k] = (k == 0) ? 0.0 : ((k <= nb) ? b[(long)r * (nb + 1) + k] / (2.0 * bi) : 0.5);
    z1[0] = 1.0;
    for (int m = 0; m < n_exp; ++m) {
        double zn[LM + 1];
#pragma unroll
        for (int k = 0; k <= LM; ++k) {
            double lower = (k > 0) ? z1[k > 0 ? k - 1 : 0] : 0.0;
            double upper = (k < LM) ? z1[k < LM ? k + 1 : LM] : 0.0;
            double full = 2.0 * (ah[k] * z1[k] + bh[k] * lower + bh[k + 1] * upper) - z0[k];
            double delay = 2.0 * bh[k] * lower;
            zn[k] = (k < L) ? full : ((k == L) ? delay : 0.0);
        }
#pragma unroll
        for (int k = 0; k <= LM; ++k) { z0[k] = z1[k]; z1[k] = zn[k]; }
        const int mm = m + 1;
        if (mm > n_mom) {
            double v = s_g[mm] * z1[0];
            gs[(long)mm * n_rows + r] = v;
            big = fmax(big, fabs(v));
        }
    }
    if (!(big <= 1e4)) flags[r] |= BOP_FLAG_DIVERGENT;
}

// ---------------------------------------------------------------------------
// per-orbital sums at energy E
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double *s_red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += s_red[q];
    __syncthreads();
    return t;    // valid in thread 0
}

// Block sums of N values per thread at once: each wave folds its values with
// shuffles, one barrier, then thread p < N adds the waves' values in wave
// order (the same additions, in the same order, as N separate block_sum calls).
// Result valid in thread p for value p.
template <int N>
__device__ inline double block_sum_n(double (&v)[N], double *s_red /* N x (DT / 64) */)
{
    constexpr int NW = DT / 64;
#pragma unroll
    for (int j = 0; j < N; ++j)
        for (int o = 32; o > 0; o >>= 1) v[j] += __shfl_xor(v[j], o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) s_red[j * NW + w] = v[j];
    }
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < N)
        for (int q = 0; q < NW; ++q) t += s_red[threadIdx.x * NW + q];
    __syncthreads();
    return t;
}

// Fermi search state: bracket [lo, hi], done flag, halvings taken so far.
struct FermiState { double lo, hi, done, halvings; };

__global__ void __launch_bounds__(DT)
k_bracket(int n_rows, const double *__restrict__ a_inf, const double *__restrict__ b_inf,
          double *__restrict__ part)
{
    __shared__ double s_lo[DT / 64], s_hi[DT / 64];
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    if (r < n_rows) { lo = a_inf[r] - 2.0 * b_inf[r]; hi = a_inf[r] + 2.0 * b_inf[r]; }
    for (int o = 32; o > 0; o >>= 1) { lo = fmin(lo, __shfl_xor(lo, o)); hi = fmax(hi, __shfl_xor(hi, o)); }
    if ((threadIdx.x & 63) == 0) { s_lo[threadIdx.x >> 6] = lo; s_hi[threadIdx.x >> 6] = hi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < DT / 64; ++q) { lo = fmin(lo, s_lo[q]); hi = fmax(hi, s_hi[q]); }
        part[2 * blockIdx.x] = lo;
        part[2 * blockIdx.x + 1] = hi;
    }
}

// The bracket from the block partials (one block, fixed order).  Global sums
// and extrema are finished in a launch of their own: a last-block scheme
// would need a device-scope fence in every block, which writes back L2.
__global__ void __launch_bounds__(DT)
k_bracket_pick(unsigned n_blocks, const double *__restrict__ part, FermiState *st)
{
    __shared__ double s_red[DT / 64];
    const double L = partials_combine(part, n_blocks, 2, 0, 1, s_red);
    const double H = partials_combine(part, n_blocks, 2, 1, 2, s_red);
    if (threadIdx.x == 0) {
        st->lo = L;
        st->hi = H;
        st->done = 0.0;
        st->halvings = 0.0;
    }
}

// Fermi level by bisection (Sec. II), four halvings per pass: the pass
// evaluates the electron count at the 15 midpoints the next four halvings can
// visit (a binary tree whose nodes are formed exactly as sequential bisection
// forms them, mid = (lo + hi)/2), reading each orbital's coefficients once;
// a one-block launch then replays the four decisions.  The decisions, and
// hence the root found when the count is not monotone, are those of plain
// bisection.
constexpr int FT_LEVELS = 4, FT_NODES = (1 << FT_LEVELS) - 1;
constexpr int FT_MAX_HALVINGS = 64;                           // as many as plain bisection takes at most
constexpr int FT_PASSES = (FT_MAX_HALVINGS + FT_LEVELS - 1) / FT_LEVELS;

__device__ inline void tree_points(double lo, double hi, double *mid)
{
    // node i (1-based, heap order) covers [l_i, h_i]; children split at mid_i
    double l[FT_NODES + 1], h[FT_NODES + 1];
    l[1] = lo;
    h[1] = hi;
#pragma unroll
    for (int i = 1; i <= FT_NODES; ++i) {
        mid[i - 1] = 0.5 * (l[i] + h[i]);
        if (2 * i + 1 <= FT_NODES) {
            l[2 * i] = l[i]; h[2 * i] = mid[i - 1];
            l[2 * i + 1] = mid[i - 1]; h[2 * i + 1] = h[i];
        }
    }
}

// Two lanes share an orbital row: lane h of the pair takes nodes 8h .. 8h+7
// (the last lane 7 nodes), which halves the registers per lane and doubles
// the rows' loads in flight; both lanes read the same coefficients.
constexpr int FT_HALF = (FT_NODES + 1) / 2;

__global__ void __launch_bounds__(DT)
k_fermi_tree(int n_rows, int n_exp, const double *__restrict__ gs, const double *__restrict__ a_inf,
             const double *__restrict__ b_inf, double *__restrict__ part, const FermiState *st)
{
    __shared__ double s_inv[1040], s_red[FT_NODES * (DT / 64)];
    if (st->done != 0.0) return;
    const double lo = st->lo, hi = st->hi;
    for (int k = threadIdx.x; k <= n_exp + 2; k += blockDim.x) s_inv[k] = k ? 1.0 / k : 0.0;
    __syncthreads();
    const long gt = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = (int)(gt >> 1), h = (int)(gt & 1);
    double cnt[FT_HALF];
    if (r < n_rows) {
        const double ai = a_inf[r], bi = b_inf[r];
        // only 2 cos(theta) and the two Clenshaw terms per node stay live in
        // the loop (the midpoints, sin(theta) and the arccos term are formed
        // before and after it), which keeps the kernel's registers low
        double twoc[FT_HALF], b1[FT_HALF], b2[FT_HALF];
        {
            double mid[FT_NODES];
            tree_points(lo, hi, mid);
#pragma unroll
            for (int j = 0; j < FT_HALF; ++j) {
                const int p = h * FT_HALF + j < FT_NODES ? h * FT_HALF + j : FT_NODES - 1;
                double eps = (mid[p] - ai) / (2.0 * bi);
                twoc[j] = 2.0 * (eps < -1.0 ? -1.0 : (eps > 1.0 ? 1.0 : eps));
                b1[j] = 0.0;
                b2[j] = 0.0;
            }
        }
        // sum_k w_k sin(k theta) = sin(theta) sum_k w_k U_(k-1)(cos theta), by
        // Clenshaw's recurrence from the highest term down; w_k = (g_(k-2) - g_k) / k
        // (w_1 = -g_1), with g_k = 0 beyond n_exp
        double gk = 0.0, gkm1 = 0.0;
#pragma unroll 4
        for (int k = n_exp + 2; k >= 1; --k) {
            const double gkm2 = (k >= 2) ? gs[(long)(k - 2) * n_rows + r] : 0.0;
            const double wk = ((k >= 2) ? (gkm2 - gk) : -gk) * s_inv[k];
            gk = gkm1;
            gkm1 = gkm2;
#pragma unroll
            for (int j = 0; j < FT_HALF; ++j) {
                const double bn = fma(twoc[j], b1[j], wk - b2[j]);
                b2[j] = b1[j];
                b1[j] = bn;
            }
        }
        const double g0 = gs[r];
#pragma unroll
        for (int j = 0; j < FT_HALF; ++j) {
            const double c = 0.5 * twoc[j];
            const double sn = sqrt(fmax(0.0, 1.0 - c * c));
            cnt[j] = g0 * (1.0 - acos(c) / M_PI) + sn * b1[j] / M_PI;
        }
    } else {
#pragma unroll
        for (int j = 0; j < FT_HALF; ++j) cnt[j] = 0.0;
    }
    {
        double v[FT_NODES];
#pragma unroll
        for (int p = 0; p < FT_NODES; ++p) v[p] = (h == p / FT_HALF) ? cnt[p % FT_HALF] : 0.0;
        const double t = block_sum_n<FT_NODES>(v, s_red);
        if (threadIdx.x < FT_NODES) part[(size_t)FT_NODES * blockIdx.x + threadIdx.x] = t;
    }
}

// The pass's decisions, in a launch of its own (one block) so that no block
// of the pass needs a device-scope fence: the block partials of every node
// are summed in a fixed order (thread t takes blocks t, t + DT, ..., then the
// fixed wave tree), and the four decisions are replayed (count < n_elec:
// lo = mid, else hi = mid), stopping when a midpoint equals an end of its
// bracket or after the most halvings plain bisection takes.
__global__ void __launch_bounds__(DT)
k_fermi_pick(unsigned n_blocks, double n_elec, const double *__restrict__ part, FermiState *st)
{
    __shared__ double s_red[FT_NODES * (DT / 64)], s_tot[FT_NODES];
    if (st->done != 0.0) return;
    const double lo = st->lo, hi = st->hi;
    double acc[FT_NODES];
#pragma unroll
    for (int p = 0; p < FT_NODES; ++p) acc[p] = 0.0;
    for (unsigned q = threadIdx.x; q < n_blocks; q += blockDim.x)
#pragma unroll
        for (int p = 0; p < FT_NODES; ++p) acc[p] += part[(size_t)q * FT_NODES + p];
    const double t = block_sum_n<FT_NODES>(acc, s_red);
    if (threadIdx.x < FT_NODES) s_tot[threadIdx.x] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[FT_NODES];
#pragma unroll
        for (int p = 0; p < FT_NODES; ++p) tot[p] = s_tot[p];
        double mid[FT_NODES];
        tree_points(lo, hi, mid);
        double l = lo, hh = hi;
        int node = 1;
        double nh = st->halvings;
        for (int lev = 0; lev < FT_LEVELS; ++lev) {
            const double m = mid[node - 1];
            if (nh >= FT_MAX_HALVINGS || m <= l || m >= hh) { st->done = 1.0; break; }
            if (2.0 * tot[node - 1] < n_elec) { l = m; node = 2 * node + 1; }
            else { hh = m; node = 2 * node; }
            nh += 1.0;
        }
        st->lo = l;
        st->hi = hh;
        st->halvings = nh;
    }
}

__global__ void k_fermi_finish(FermiState *st, double *E_F)
{
    E_F[0] = 0.5 * (st->lo + st->hi);
}

// per-atom N, U, n(E_F) and block partials of U.  One thread per orbital row
// (EA atoms x n_orb rows per block, so the GPU has enough waves for the long
// per-row sums); an atom's orbitals are then added in orbital order, as a
// per-atom loop would add them.
constexpr int EA = 64;           // atoms per block of the energy pass

__global__ void __launch_bounds__(EA * 9)
k_energy(int n_atoms, int no, int n_exp, double wt, const double *__restrict__ gs, const double *__restrict__ a_inf,
         const double *__restrict__ b_inf, const double *__restrict__ H_on, const double *__restrict__ E_F,
         double *__restrict__ N_atom, double *__restrict__ U_atom, double *__restrict__ dos_atom,
         int *__restrict__ flags, double *__restrict__ part)
{
    __shared__ double s_inv[1040], s_red[EA * 9 / 64], s_n[EA * 9], s_u[EA * 9], s_d[EA * 9];
    for (int k = threadIdx.x; k <= n_exp + 4; k += blockDim.x) s_inv[k] = k ? 1.0 / k : 0.0;
    __syncthreads();
    const double E = E_F[0];
    const long n_rows = (long)n_atoms * no;
    const long r = (long)blockIdx.x * EA * no + threadIdx.x;
    double N = 0.0, U = 0.0, D = 0.0;
    if (r < n_rows) {
        double ai = a_inf[r], bi = b_inf[r];
        double eps = (E - ai) / (2.0 * bi);
        double c = eps < -1.0 ? -1.0 : (eps > 1.0 ? 1.0 : eps);
        double s = sqrt(fmax(0.0, 1.0 - c * c));
        double phi = acos(c);
        // sin((m+1) phi), sin((m+2) phi) and (cos, sin)((m+3) phi), advanced
        // by unit-modulus rotation; chi^_m, chi^_(m+1) carried along
        const double c2 = c * c - s * s, s2 = 2.0 * c * s;
        double w1 = s, w2 = s2;
        double c3 = c2 * c - s2 * s, w3 = s2 * c + c2 * s;
        double chi0 = 0.0;
        double chi1 = 1.0 - phi / M_PI + s2 / (2.0 * M_PI);
#pragma unroll 8
        for (int m = 0; m <= n_exp; ++m) {
            // chi^_(m+2) = (sin((m+3) phi)/(m+3) - sin((m+1) phi)/(m+1)) / pi
            double chi2 = (w3 * s_inv[m + 3] - w1 * s_inv[m + 1]) / M_PI;
            double g = gs[(long)m * n_rows + r];
            N = fma(g, chi1, N);
            U = fma(g, chi2 + chi0, U);
            D = fma(g, w1, D);
            chi0 = chi1;
            chi1 = chi2;
            double nc = c3 * c - w3 * s, ns = w3 * c + c3 * s;
            w1 = w2; w2 = w3; w3 = ns; c3 = nc;
        }
        U = bi * U + (ai - H_on[r]) * N;
        D = (eps > -1.0 && eps < 1.0) ? D / (M_PI * bi) : 0.0;
        if (!(eps > -1.0 && eps < 1.0)) flags[r] |= BOP_FLAG_OUTSIDE;
    }
    s_n[threadIdx.x] = N;
    s_u[threadIdx.x] = U;
    s_d[threadIdx.x] = D;
    __syncthreads();
    const int t = threadIdx.x;
    const long i = (long)blockIdx.x * EA + t;
    double Ui = 0.0;
    if (t < EA && i < n_atoms) {
        double sN = 0.0, sU = 0.0, sD = 0.0;
        for (int a = 0; a < no; ++a) {
            sN += s_n[t * no + a];
            sU += s_u[t * no + a];
            sD += s_d[t * no + a];
        }
        // both spins; wt orbitals per row in the atom-averaged mode
        N_atom[i] = 2.0 * wt * sN;
        U_atom[i] = 2.0 * wt * sU;
        dos_atom[i] = 2.0 * wt * sD;
        Ui = 2.0 * wt * sU;
    }
    const double tb = block_sum(Ui, s_red);
    if (threadIdx.x == 0) part[blockIdx.x] = tb;
}

// total U from the block partials (one block, fixed order)
__global__ void __launch_bounds__(DT)
k_energy_total(unsigned n_blocks, const double *__restrict__ part, double *__restrict__ U_total)
{
    __shared__ double s_red[DT / 64];
    const double tot = partials_combine(part, n_blocks, 1, 0, 0, s_red);
    if (threadIdx.x == 0) U_total[0] = tot;
}

struct EnergyWs {
    double *gs, *part;
    FermiState *st;
    size_t bytes;
};

EnergyWs carve(void *base, long n_rows, int n_exp)
{
    EnergyWs w{};
    char *p = (char *)base;
    auto take = [&](size_t b) { char *r = p; p += align_up(b, 256); return (void *)r; };
    w.gs = (double *)take(sizeof(double) * (size_t)(n_exp + 1) * (size_t)n_rows);
    long nblk = 2 * ((n_rows + DT - 1) / DT) + 1;       // two lanes per row in the Fermi passes
    w.part = (double *)take(sizeof(double) * FT_NODES * (size_t)nblk);
    w.st = (FermiState *)take(sizeof(FermiState));
    w.bytes = (size_t)(p - (char *)base);
    return w;
}

}  // namespace
}  // namespace bop

using namespace bop;

extern "C" int bop_recursion(int n_rows, int n_max, const double *mu, int bw_mode, double a_glob,
                             double b_glob, double *a, double *b, double *a_inf, double *b_inf,
                             int *flags, hipStream_t stream)
{
    BOP_REQUIRE(n_rows >= 0, BOP_E_ARG, "bop_recursion: n_rows < 0");
    BOP_REQUIRE(n_max >= 1 && n_max <= MAX_NMAX, BOP_E_UNSUPPORTED, "bop_recursion: n_max must be 1..%d", MAX_NMAX);
    BOP_REQUIRE(bw_mode >= BOP_BW_GERSHGORIN && bw_mode <= BOP_BW_WEIGHTED, BOP_E_ARG,
                "bop_recursion: bw_mode must be %d..%d", BOP_BW_GERSHGORIN, BOP_BW_WEIGHTED);
    BOP_REQUIRE(bw_mode != BOP_BW_WEIGHTED || a_glob >= 0.0, BOP_E_ARG, "bop_recursion: weighted beta must be >= 0");
    if (n_rows == 0) return BOP_OK;
    BOP_REQUIRE(a && b && a_inf && b_inf && flags, BOP_E_ARG, "bop_recursion: NULL array");
    // the register kernel covers Gershgorin and the global values; the other
    // estimates read the chain back from a and b in the generic kernel
    if (mu && n_max <= 20 && bw_mode <= BOP_BW_GLOBAL)
        k_recursion_reg<20><<<(n_rows + DT - 1) / DT, DT, 0, stream>>>(n_rows, n_max, mu, bw_mode, a_glob, b_glob,
                                                                       a, b, a_inf, b_inf, flags);
    else
    k_recursion<<<(n_rows + DT - 1) / DT, DT, 0, stream>>>(n_rows, n_max, mu, bw_mode, a_glob, b_glob, a, b,
                                                           a_inf, b_inf, flags);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" size_t bop_energy_workspace_size(int n_atoms, int n_orb, int n_exp)
{
    if (n_atoms < 0 || n_orb <= 0 || n_exp < 0) return 0;
    return carve(nullptr, (long)n_atoms * n_orb, n_exp).bytes + 256;
}

// wt: orbitals each row stands for (1; n_orb in the atom-averaged mode, where
// a row is an atom's averaged chain): the Fermi search counts wt 2 N per row
// and the per-atom outputs are scaled by wt.
static int energy_impl(int n_atoms, int no, int n_max, int n_exp, const double *mu, const double *a,
                       const double *b, const double *a_inf, const double *b_inf, const double *H_on,
                       double n_elec, int ef_mode, double *E_F, double *N_atom, double *U_atom,
                       double *dos_atom, double *U_total, int *flags, void *ws, size_t ws_bytes,
                       hipStream_t stream, double wt = 1.0)
{
    BOP_REQUIRE(n_atoms > 0 && no > 0, BOP_E_ARG, "bop_energy: n_atoms and n_orb must be > 0");
    BOP_REQUIRE(no <= 9, BOP_E_UNSUPPORTED, "bop_energy: at most 9 orbitals per atom");
    BOP_REQUIRE(n_max >= 1 && n_max <= MAX_NMAX, BOP_E_UNSUPPORTED, "bop_energy: n_max must be 1..%d", MAX_NMAX);
    BOP_REQUIRE(n_exp >= 1 && n_exp <= 1024, BOP_E_UNSUPPORTED, "bop_energy: n_exp must be 1..1024");
    BOP_REQUIRE(ef_mode == 0 || ef_mode == 1, BOP_E_ARG, "bop_energy: ef_mode must be 0 or 1");
    BOP_REQUIRE(a && b && a_inf && b_inf && H_on && E_F && N_atom && U_atom && dos_atom && U_total && flags,
                BOP_E_ARG, "bop_energy: NULL array");
    const long R = (long)n_atoms * no;
    EnergyWs w = carve(ws, R, n_exp);
    BOP_REQUIRE(ws && ws_bytes >= w.bytes, BOP_E_CAPACITY, "bop_energy: workspace of %zu bytes needed", w.bytes);
    BOP_REQUIRE(ef_mode == 1 || (n_elec >= 0.0 && n_elec <= 2.0 * wt * (double)R), BOP_E_ARG,
                "bop_energy: n_elec outside [0, 2 n_rows]");
    const unsigned nblk = (unsigned)((R + DT - 1) / DT);
    const int L = (n_max - 1) / 2 + 1 > n_max / 2 ? (n_max - 1) / 2 + 1 : n_max / 2;
    if (L <= 11) k_dos_coeffs<11><<<nblk, DT, 0, stream>>>((int)R, n_max, n_exp, mu, a, b, a_inf, b_inf, w.gs, flags);
    else k_dos_coeffs<21><<<nblk, DT, 0, stream>>>((int)R, n_max, n_exp, mu, a, b, a_inf, b_inf, w.gs, flags);
    BOP_LAUNCHED();
    if (ef_mode == 0) {
        k_bracket<<<nblk, DT, 0, stream>>>((int)R, a_inf, b_inf, w.part);
        k_bracket_pick<<<1, DT, 0, stream>>>(nblk, w.part, w.st);
        BOP_LAUNCHED();
        const unsigned fblk = (unsigned)((2 * R + DT - 1) / DT);
        for (int it = 0; it < FT_PASSES; ++it) {
            k_fermi_tree<<<fblk, DT, 0, stream>>>((int)R, n_exp, w.gs, a_inf, b_inf, w.part, w.st);
            k_fermi_pick<<<1, DT, 0, stream>>>(fblk, n_elec / wt, w.part, w.st);
        }
        BOP_LAUNCHED();
        k_fermi_finish<<<1, 1, 0, stream>>>(w.st, E_F);
        BOP_LAUNCHED();
    }
    const unsigned ablk = (unsigned)((n_atoms + EA - 1) / EA);
    k_energy<<<ablk, EA * no, 0, stream>>>(n_atoms, no, n_exp, wt, w.gs, a_inf, b_inf, H_on, E_F, N_atom, U_atom,
                                      dos_atom, flags, w.part);
    k_energy_total<<<1, DT, 0, stream>>>(ablk, w.part, U_total);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" int bop_energy(int n_atoms, int no, int n_max, int n_exp, const double *mu, const double *a,
                          const double *b, const double *a_inf, const double *b_inf, const double *H_on,
                          double n_elec, int ef_mode, double *E_F, double *N_atom, double *U_atom,
                          double *dos_atom, double *U_total, int *flags, void *ws, size_t ws_bytes,
                          hipStream_t stream)
{
    return energy_impl(n_atoms, no, n_max, n_exp, mu, a, b, a_inf, b_inf, H_on, n_elec, ef_mode, E_F, N_atom,
                       U_atom, dos_atom, U_total, flags, ws, ws_bytes, stream);
}

// Atom-averaged mode: one chain per atom from mu_i / n_orb.
__global__ void __launch_bounds__(DT)
k_atom_average(int n_atoms, int no, int n_max, const double *__restrict__ mu, const double *__restrict__ H_on,
               double *__restrict__ mu_avg, double *__restrict__ H_avg)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int M = n_max + 1;
    if (e >= (long)n_atoms * M) return;
    const long i = e / M;
    const int n = (int)(e % M);
    double s = 0.0;
    for (int a = 0; a < no; ++a) s += mu[(i * no + a) * M + n];
    mu_avg[e] = s / no;
    if (n == 0) {
        double h = 0.0;
        for (int a = 0; a < no; ++a) h += H_on[i * no + a];
        H_avg[i] = h / no;
    }
}

extern "C" int bop_atom_average(int n_atoms, int n_orb, int n_max, const double *mu, const double *H_on,
                                double *mu_avg, double *H_avg, hipStream_t stream)
{
    BOP_REQUIRE(n_atoms >= 0 && n_orb > 0 && n_max >= 0 && n_max <= MAX_NMAX, BOP_E_ARG,
                "bop_atom_average: bad sizes");
    if (n_atoms == 0) return BOP_OK;
    BOP_REQUIRE(mu && H_on && mu_avg && H_avg, BOP_E_ARG, "bop_atom_average: NULL array");
    const long ne = (long)n_atoms * (n_max + 1);
    k_atom_average<<<(unsigned)((ne + DT - 1) / DT), DT, 0, stream>>>(n_atoms, n_orb, n_max, mu, H_on, mu_avg, H_avg);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" int bop_energy_atom_averaged(int n_atoms, int n_orb, int n_max, int n_exp, const double *mu_avg,
                                        const double *a, const double *b, const double *a_inf,
                                        const double *b_inf, const double *H_avg, double n_elec, int ef_mode,
                                        double *E_F, double *N_atom, double *U_atom, double *dos_atom,
                                        double *U_total, int *flags, void *ws, size_t ws_bytes, hipStream_t stream)
{
    BOP_REQUIRE(n_orb > 0, BOP_E_ARG, "bop_energy_atom_averaged: n_orb must be > 0");
    return energy_impl(n_atoms, 1, n_max, n_exp, mu_avg, a, b, a_inf, b_inf, H_avg, n_elec, ef_mode, E_F, N_atom,
                       U_atom, dos_atom, U_total, flags, ws, ws_bytes, stream, (double)n_orb);
}

// ---------------------------------------------------------------------------
// bop_energy without a caller workspace: the expansion coefficients, block
// partials and Fermi state live in a fixed device array of
// BOP_ENERGY_NOALLOC_BYTES, one copy per GPU the library runs on, held until
// the process ends.  Nothing in it must start at zero: every kernel writes the
// part of the workspace it reads before reading it.  Calls that overlap on one
// GPU (several streams or threads) share the array and race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[BOP_ENERGY_NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES];     // the array's device address on each GPU (NULL: not looked up yet)
}  // namespace

// The device address of `scratch` on the current GPU, looked up once per GPU
// with that GPU current.  The array's name in host code is only a host-side
// handle, never a device address.
static int scratch_address(void **out)
{
    int dev = -1;
    BOP_HIP(hipGetDevice(&dev));
    BOP_REQUIRE(dev >= 0 && dev < MAX_DEVICES, BOP_E_UNSUPPORTED, "bop_energy_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        BOP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        BOP_REQUIRE(p, BOP_E_HIP, "bop_energy_noalloc: no device address for the scratch array");
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return BOP_OK;
}

extern "C" int bop_energy_noalloc(int n_atoms, int no, int n_max, int n_exp, const double *mu, const double *a,
                                  const double *b, const double *a_inf, const double *b_inf, const double *H_on,
                                  double n_elec, int ef_mode, double *E_F, double *N_atom, double *U_atom,
                                  double *dos_atom, double *U_total, int *flags, hipStream_t stream)
{
    BOP_REQUIRE(n_atoms > 0 && no > 0 && n_exp >= 0, BOP_E_ARG, "bop_energy_noalloc: n_atoms and n_orb must be > 0");
    const size_t need = carve(nullptr, (long)n_atoms * no, n_exp).bytes;
    BOP_REQUIRE(need <= BOP_ENERGY_NOALLOC_BYTES, BOP_E_CAPACITY,
                "bop_energy_noalloc: %d atoms x %d orbitals at n_exp %d need %zu bytes of scratch, more than its "
                "fixed %llu; use bop_energy with a caller workspace",
                n_atoms, no, n_exp, need, (unsigned long long)BOP_ENERGY_NOALLOC_BYTES);
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != BOP_OK) return rc;
    return energy_impl(n_atoms, no, n_max, n_exp, mu, a, b, a_inf, b_inf, H_on, n_elec, ef_mode, E_F, N_atom,
                       U_atom, dos_atom, U_total, flags, ws, BOP_ENERGY_NOALLOC_BYTES, stream);
}

namespace bop {
double *energy_ws_scratch(void *ws, long n_rows, int n_exp)
{
    return carve(ws, n_rows, n_exp).part;
}
}  // namespace bop
