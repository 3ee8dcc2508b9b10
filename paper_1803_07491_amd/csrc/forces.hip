// Forces of the d-band bond energy (App. C.1-C.2 of arXiv:1803.07491): the
// general derivative dU/dLambda through the weights w = dU/dmu (Eqs.
// dUdLambda, weights), the bond-order-like Theta~ = dU/dH (Eqs. theta-tilde,
// Theta_tilde_BOP) and F_k = -sum Theta~ grad_k H (Eq. F_k).
//
//  * Weights: each orbital's energy tail (recursion with the Gershgorin
//    terminator, Chebyshev coefficients from the moments and from the
//    terminated chain, Jackson damping, N and U at E_F) in forward-mode dual
//    numbers, one moment (derivative direction) per thread.  The Fermi level
//    follows the moments to keep the electron count, which adds
//    -(E_F - E_bar) dN/dmu to dU/dmu, E_bar = sum e_r n_r(E_F) / sum n_r(E_F)
//    (dE_F/dmu = -(dN/dmu) / n(E_F); dU/dE_F = (E_F - e_r) n_r(E_F)).
//  * Theta~ per tile of 64 columns (the moment tiles: atoms' orbitals as
//    columns).  With X^l = H^l e_c and the transfer vectors
//        G^k = w_k e_c + H G^(k+1),   G^(n+1) = 0
//    (the transfer-path recursion T^(n,m) = H T^(n-1,m) + w xi^(n), summed
//    over m by Horner's rule), dU = sum_c sum_(k=1..n) <G_c^k, dH X_c^(k-1)>,
//    so Theta~_(i a, j b) = sum_c sum_(k=0..n-1) X_c^k[i a] G_c^(k+1)[j b]
//    (the two ends of a path swap by the transpose property; per column the
//    sum is symmetric in (i a) <-> (j b)).
//    X^l is non-zero within l hops of the tile and is needed only within
//    n - l hops (G^(l+1) vanishes beyond n - l - 1), and likewise G^k, so
//    both are formed on the atoms within min(l, n - l) <= n/2 hops: the
//    moment plan's support, whose layers order the rows and whose neighbour
//    slots are sorted by layer, so each product reads a prefix of a row's
//    slots.  Every value formed this way is exact: a product at a row of
//    layer L reads neighbours of layers up to L + 1 only where the operand
//    is kept there, and the operand vanishes where it is not.
//  * Forward passes store X^0 .. X^(n-1) (level l on layers <= min(l, n-l));
//    backward passes k = n-1 .. 0 form G^k at each row (one wave per row, a
//    lane per column) from the gathered G^(k+1) of its neighbours and, with
//    the same gathers and the row's own X^k, the per-pair contraction
//    sum_(a,b) X^k[i a] G^(k+1)[j b] dH_(ij,ab)/dd, summed over the 64 columns
//    by a wave reduction.  A pair's partial sums live in a per-tile slot
//    array from the row's first backward pass (k = n - L) to its last
//    (k = L), where they are added to the pair's gradient with one FP64
//    atomic per component.  Per column the sum is symmetric and the block
//    derivatives of the two directions of a bond are transposes of opposite
//    sign, so g_reverse(p) = -g_p: only the direction with the lower pair
//    index is contracted, and stored doubled.
//  * Bond-block derivatives: the d-d block as V_sigma P_sigma + V_pi P_pi +
//    V_delta P_delta with projectors built from the real d harmonics Y(u) of
//    the bond direction u: P_sigma = Y Y^T, P_pi = (sum_x dY/du_x dY/du_x^T -
//    4 P_sigma) / 3, P_delta = 1 - P_sigma - P_pi (the two-centre blocks of
//    App. A.2.1 written without angles, so smooth on the polar axis), in dual
//    numbers of the three components of the bond vector.
//  * F_k = sum over k's pairs p of g_p - g_(reverse of p), with g_p =
//    sum_ab Theta~_p,ab dH_p,ab/dd_p (d_p = r_j + S - r_i); with the doubled
//    canonical direction and a zero reverse this is the same sum.
#include "bop_internal.h"
#include "tiles.h"

#include <cmath>

namespace bop {
namespace {

constexpr int FW = 256;             // threads per block of the force passes
constexpr int NWF = FW / 64;
// Rows per chunk of the force passes, independent of the moment plan's: a
// tile's chunks then fill about one XCD, so about one tile's rows are in
// flight per XCD and its gathered FP64 rows stay in that XCD's L2, where
// larger chunks put several tiles' windows in one L2.
constexpr int F_CHUNK = 16;
constexpr int WT = 256;             // threads per block of the weight kernels
constexpr int F_MAXN = 20;          // largest n_max of the force path

// ---------------------------------------------------------------------------
// forward-mode dual numbers: value and N partial derivatives
// ---------------------------------------------------------------------------
template <int N>
struct Dual {
    double v;
    double d[N];
};

template <int N> __device__ inline Dual<N> dc(double v)
{
    Dual<N> r;
    r.v = v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = 0.0;
    return r;
}
template <int N> __device__ inline Dual<N> operator+(const Dual<N> &a, const Dual<N> &b)
{
    Dual<N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = a.d[q] + b.d[q];
    return r;
}
template <int N> __device__ inline Dual<N> operator-(const Dual<N> &a, const Dual<N> &b)
{
    Dual<N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = a.d[q] - b.d[q];
    return r;
}
template <int N> __device__ inline Dual<N> operator-(const Dual<N> &a)
{
    Dual<N> r;
    r.v = -a.v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = -a.d[q];
    return r;
}
template <int N> __device__ inline Dual<N> operator*(const Dual<N> &a, const Dual<N> &b)
{
    Dual<N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = a.d[q] * b.v + a.v * b.d[q];
    return r;
}
template <int N> __device__ inline Dual<N> operator*(double s, const Dual<N> &a)
{
    Dual<N> r;
    r.v = s * a.v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = s * a.d[q];
    return r;
}
template <int N> __device__ inline Dual<N> operator*(const Dual<N> &a, double s) { return s * a; }
template <int N> __device__ inline Dual<N> operator+(const Dual<N> &a, double s)
{
    Dual<N> r = a;
    r.v += s;
    return r;
}
template <int N> __device__ inline Dual<N> operator+(double s, const Dual<N> &a) { return a + s; }
template <int N> __device__ inline Dual<N> operator-(const Dual<N> &a, double s) { return a + (-s); }
template <int N> __device__ inline Dual<N> operator-(double s, const Dual<N> &a) { return (-a) + s; }
template <int N> __device__ inline Dual<N> operator/(const Dual<N> &a, const Dual<N> &b)
{
    Dual<N> r;
    r.v = a.v / b.v;
    const double ib = 1.0 / b.v;
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = (a.d[q] - r.v * b.d[q]) * ib;
    return r;
}
template <int N> __device__ inline Dual<N> operator/(const Dual<N> &a, double s) { return (1.0 / s) * a; }
template <int N> __device__ inline Dual<N> dsqrt(const Dual<N> &a)
{
    Dual<N> r;
    r.v = sqrt(a.v);
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = a.d[q] / (2.0 * r.v);
    return r;
}
// arccos of c in (-1, 1), given s = sqrt(1 - c^2) > 0
template <int N> __device__ inline Dual<N> dacos(const Dual<N> &c, double s)
{
    Dual<N> r;
    r.v = acos(c.v);
#pragma unroll
    for (int q = 0; q < N; ++q) r.d[q] = -c.d[q] / s;
    return r;
}

// ---------------------------------------------------------------------------
// weights: dU/dmu and dN/dmu per (orbital row, moment) at E_F
// ---------------------------------------------------------------------------
__device__ inline int fa_of(int n_max) { return n_max >= 1 ? (n_max - 1) / 2 + 1 : 0; }
__device__ inline int fb_of(int n_max) { return n_max / 2; }

// One thread per (row, direction dir = 1..n_max): the row's tail with the
// normalised moments seeded by d m_t / d mu_dir = [t = dir] / mu_0.  The
// branch decisions (breakdown, band edges, width floor, inside the band) are
// taken on the values.  Writes dU, dN [R][n_max + 1] (column 0 untouched) and,
// from the dir = 1 thread, n_r(E_F) of the row.
// Two waves per SIMD: unbounded, the compiler takes all 256 VGPRs and runs
// one; bounded to four it spills the chain.
template <int LM>
__global__ void __launch_bounds__(WT) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_weights(int R, int n_max, int n_exp, const double *__restrict__ mu, const double *__restrict__ H_on,
          const double *__restrict__ E_F, double *__restrict__ dU, double *__restrict__ dN, double *__restrict__ Drow)
{
    using D1 = Dual<1>;
    __shared__ double s_p[(F_MAXN + 1) * (F_MAXN + 1)];   // coefficients of U_m in powers of x
    __shared__ double s_c[(F_MAXN + 1) * (F_MAXN + 1)];   // binomials
    __shared__ double s_g[1025];                          // Jackson factors for U_m
    __shared__ double s_inv[1030];
    const int M = n_max + 1;
    if (threadIdx.x == 0) {
        for (int t = 0; t < M * M; ++t) { s_p[t] = 0.0; s_c[t] = 0.0; }
        s_p[0] = 1.0;
        if (M > 1) s_p[M + 1] = 2.0;
        for (int m = 1; m + 1 < M; ++m)
            for (int q = 0; q <= m + 1; ++q)
                s_p[(m + 1) * M + q] = (q >= 1 ? 2.0 * s_p[m * M + q - 1] : 0.0) - (q <= m - 1 ? s_p[(m - 1) * M + q] : 0.0);
        for (int q = 0; q < M; ++q) {
            s_c[q * M] = 1.0;
            for (int l = 1; l <= q; ++l) s_c[q * M + l] = s_c[(q - 1) * M + l - 1] + (l <= q - 1 ? s_c[(q - 1) * M + l] : 0.0);
        }
    }
    {
        const double wj = M_PI / (n_exp + 1.0);
        const double cotw = cos(wj) / sin(wj);
        const double g1 = ((double)n_exp * cos(wj) + sin(wj) * cotw) / (n_exp + 1.0);
        for (int m = threadIdx.x; m <= n_exp; m += blockDim.x) {
            const int mm = m + 1;
            s_g[m] = (((double)(n_exp - mm + 1) * cos(wj * mm) + sin(wj * mm) * cotw) / (n_exp + 1.0)) / g1;
        }
        for (int k = threadIdx.x; k <= n_exp + 4; k += blockDim.x) s_inv[k] = k ? 1.0 / k : 0.0;
    }
    __syncthreads();
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long r = tid / n_max;
    const int dir = 1 + (int)(tid % n_max);
    if (r >= R) return;
    const int na = fa_of(n_max), nb = fb_of(n_max);
    const double *mr = mu + r * M;
    const double m0 = mr[0];
    D1 m[F_MAXN + 1];
    for (int t = 0; t < M; ++t) {
        m[t] = dc<1>(mr[t] / m0);
        m[t].d[0] = (t == dir) ? 1.0 / m0 : 0.0;
    }
    // recursion coefficients from the moments (orthonormal polynomials by
    // their coefficients in powers of H)
    D1 a[F_MAXN / 2 + 1], b[F_MAXN / 2 + 2];
    D1 cp[F_MAXN / 2 + 3], cc[F_MAXN / 2 + 3], dv[F_MAXN / 2 + 3];
    for (int q = 0; q < F_MAXN / 2 + 3; ++q) { cp[q] = dc<1>(0.0); cc[q] = dc<1>(0.0); }
    for (int q = 0; q < F_MAXN / 2 + 2; ++q) b[q] = dc<1>(0.0);
    cc[0] = dc<1>(1.0);
    D1 bn = dc<1>(0.0);
    const double var = n_max >= 2 ? m[2].v - m[1].v * m[1].v : 0.0;
    bool broke = false;
    for (int q = 0; q < na; ++q) {
        if (broke) { a[q] = a[q - 1]; continue; }
        D1 s = dc<1>(0.0);
        for (int j = 0; j <= q; ++j)
            for (int l = 0; l <= q; ++l) s = s + cc[j] * cc[l] * m[j + l + 1];
        a[q] = s;
        if (q + 1 > nb) break;
        for (int j = 0; j <= q + 1; ++j) dv[j] = (j > 0 ? cc[j - 1] : dc<1>(0.0)) - s * cc[j] - bn * cp[j];
        D1 b2 = dc<1>(0.0);
        for (int j = 0; j <= q + 1; ++j)
            for (int l = 0; l <= q + 1; ++l) b2 = b2 + dv[j] * dv[l] * m[j + l];
        if (!(b2.v > 1e-14 * var)) {
            broke = true;
            continue;
        }
        const D1 bb = dsqrt(b2);
        b[q + 1] = bb;
        for (int j = 0; j <= q + 1; ++j) { cp[j] = cc[j]; cc[j] = dv[j] / bb; }
        bn = bb;
    }
    // Gershgorin band edges (the extremes chosen by value)
    D1 lo = dc<1>(0.0), hi = dc<1>(0.0);
    for (int q = 0; q < na; ++q) {
        const D1 bl = (q >= 1 && q <= nb) ? b[q] : dc<1>(0.0);
        const D1 bh = (q + 1 <= nb) ? b[q + 1] : dc<1>(0.0);
        const D1 e0 = a[q] - bl - bh, e1 = a[q] + bl + bh;
        if (q == 0 || e0.v < lo.v) lo = e0;
        if (q == 0 || e1.v > hi.v) hi = e1;
    }
    const D1 ai = 0.5 * (hi + lo);
    D1 bi = 0.25 * (hi - lo);
    if (!(bi.v >= 1e-6)) bi = dc<1>(1e-6);
    const int n_mom = bi.v > 1e-6 ? n_max : 0;
    // sigma_m from the moments for m <= n_mom: normalised moments of the
    // scaled variable, then the U_m coefficients
    D1 gm[F_MAXN + 1];
    if (n_mom > 0) {
        D1 mh[F_MAXN + 1];
        const D1 two_b = 2.0 * bi;
        D1 scale = dc<1>(1.0);
        for (int q = 0; q < M; ++q) {
            D1 s = dc<1>(0.0), pa = dc<1>(1.0);
            for (int l = 0; l <= q; ++l) {
                s = s + s_c[q * M + l] * (pa * m[q - l]);
                pa = pa * (-ai);
            }
            mh[q] = s / scale;
            scale = scale * two_b;
        }
        for (int q = 0; q < M; ++q) {
            D1 s = dc<1>(0.0);
            for (int l = 0; l <= q; ++l) s = s + s_p[q * M + l] * mh[l];
            gm[q] = s;
        }
    } else {
        gm[0] = dc<1>(1.0);
    }
    // chain on levels 0..L with the delay level L (the free terminated tail)
    const int L = na > nb ? na : nb;
    D1 ah[LM + 1], bh[LM + 2], z0[LM + 1], z1[LM + 1];
    const D1 tb = 2.0 * bi;
#pragma unroll
    for (int k = 0; k <= LM; ++k) {
        ah[k] = (k < na) ? (a[k < na ? k : 0] - ai) / tb : dc<1>(0.0);
        z0[k] = dc<1>(0.0);
        z1[k] = dc<1>(0.0);
    }
#pragma unroll
    for (int k = 0; k <= LM + 1; ++k)
        bh[k] = (k == 0) ? dc<1>(0.0) : ((k <= nb) ? b[k <= nb ? k : 0] / tb : dc<1>(0.5));
    z1[0] = dc<1>(1.0);
    // N, U and n(E) at E_F by the Chebyshev sums with chi functions, the
    // sines advanced by rotation
    const double E = E_F[0];
    const D1 eps = (E - ai) / tb;
    const bool inside = eps.v > -1.0 && eps.v < 1.0;
    const D1 c = inside ? eps : dc<1>(eps.v <= -1.0 ? -1.0 : 1.0);
    const double sv = sqrt(fmax(0.0, 1.0 - c.v * c.v));
    D1 sn = dc<1>(sv);
    if (inside) sn.d[0] = -c.v * c.d[0] / sv;
    const D1 phi = inside ? dacos(c, sv) : dc<1>(acos(c.v));
    const D1 c2 = c * c - sn * sn, s2 = 2.0 * (c * sn);
    D1 w1 = sn, w2 = s2;
    D1 c3 = c2 * c - s2 * sn, w3 = s2 * c + c2 * sn;
    D1 chi0 = dc<1>(0.0);
    D1 chi1 = 1.0 - phi / M_PI + s2 / (2.0 * M_PI);
    D1 N = dc<1>(0.0), U = dc<1>(0.0), Dd = dc<1>(0.0);
    // one term m of the sums, sigma_m given
    auto term = [&](int mstep, const D1 &sig) {
        const D1 g = s_g[mstep] * sig;
        const D1 chi2 = (1.0 / M_PI) * (w3 * s_inv[mstep + 3] - w1 * s_inv[mstep + 1]);
        N = N + g * chi1;
        U = U + g * (chi2 + chi0);
        Dd = Dd + g * w1;
        chi0 = chi1;
        chi1 = chi2;
        const D1 nc = c3 * c - w3 * sn, ns = w3 * c + c3 * sn;
        w1 = w2;
        w2 = w3;
        w3 = ns;
        c3 = nc;
    };
    // the chain from sigma_0 = 1 one step on: afterwards z1[0] = sigma_(m+1)
    auto advance = [&]() {
        // in place, level by level: lower holds the old z1[k - 1]
        D1 lower = dc<1>(0.0);
#pragma unroll
        for (int k = 0; k <= LM; ++k) {
            const D1 cur = z1[k];
            const D1 upper = (k < LM) ? z1[k < LM ? k + 1 : LM] : dc<1>(0.0);
            const D1 full = 2.0 * (ah[k] * cur + bh[k] * lower + bh[k + 1] * upper) - z0[k];
            const D1 delay = 2.0 * (bh[k] * lower);
            z1[k] = (k < L) ? full : ((k == L) ? delay : dc<1>(0.0));
            z0[k] = cur;
            lower = cur;
        }
    };
    // m <= n_mom: sigma_m from the moments (unrolled, so that gm is indexed
    // at compile time and dies before the chain's arrays are live)
#pragma unroll
    for (int q = 0; q <= F_MAXN; ++q)
        if (q <= n_mom && q <= n_exp) term(q, n_mom > 0 ? gm[q] : dc<1>(1.0));
    // m > n_mom: sigma_m from the chain, first advanced to sigma_(n_mom + 1)
    if (n_mom < n_exp) {
        for (int mstep = 0; mstep <= n_mom; ++mstep) advance();
        for (int mstep = n_mom + 1; mstep <= n_exp; ++mstep) {
            term(mstep, z1[0]);
            if (mstep < n_exp) advance();
        }
    }
    U = bi * U + (ai - H_on[r]) * N;
    dU[r * M + dir] = U.d[0];
    dN[r * M + dir] = N.d[0];
    if (dir == 1) Drow[r] = inside ? Dd.v / (M_PI * bi.v) : 0.0;
}

// block partials of sum e_r n_r(E_F) and sum n_r(E_F)
__global__ void __launch_bounds__(WT)
k_ebar_part(int R, const double *__restrict__ H_on, const double *__restrict__ Drow, double *__restrict__ part)
{
    __shared__ double s_red[WT / 64];
    const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const double d = r < R ? Drow[r] : 0.0;
    const double ed = r < R ? H_on[r] * d : 0.0;
    const double t1 = block_combine(ed, 0, s_red);
    const double t0 = block_combine(d, 0, s_red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = t1;
        part[2 * blockIdx.x + 1] = t0;
    }
}

__global__ void __launch_bounds__(WT)
k_ebar(unsigned n_blocks, const double *__restrict__ part, double *__restrict__ ebar)
{
    __shared__ double s_red[WT / 64];
    const double s1 = partials_combine(part, n_blocks, 2, 0, 0, s_red);
    const double s0 = partials_combine(part, n_blocks, 2, 1, 0, s_red);
    if (threadIdx.x == 0) ebar[0] = s1 / s0;
}

// w = 2 (dU - (E_F - E_bar) dN) (both spins), w[., 0] = 0
__global__ void __launch_bounds__(WT)
k_wfinish(long n, int M, const double *__restrict__ dU, const double *__restrict__ dN,
          const double *__restrict__ E_F, const double *__restrict__ ebar, double *__restrict__ w)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    w[e] = (e % M == 0) ? 0.0 : 2.0 * (dU[e] - (E_F[0] - ebar[0]) * dN[e]);
}

// ---------------------------------------------------------------------------
// bond-block derivatives dH_p / dd_p (packed symmetric, [P][3][16])
// ---------------------------------------------------------------------------
__device__ inline int pair_owner(const int *__restrict__ row_ptr, int n, long p)
{
    int lo = 0, hi = n - 1;            // largest i with row_ptr[i] <= p
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_ptr[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// bond integral and its radial derivative (Eq. cutoff taper included)
__device__ inline void bond_integral_dr(const bop_model &m, int pair, int ch, double r, double &v, double &dv)
{
    const double b0 = m.beta0[pair][ch];
    v = 0.0;
    dv = 0.0;
    if (b0 == 0.0) return;
    const double q = m.q[pair][ch], r0 = m.r0[pair][ch];
    if (m.form[pair][ch] == BOP_FORM_POWER) {
        v = b0 * pow(r0 / r, q);
        dv = -q * v / r;
    } else {
        v = b0 * exp(-q * (r - r0));
        dv = -q * v;
    }
    if (m.d_cut > 0.0 && r >= m.r_cut - m.d_cut) {
        const double x = (r - (m.r_cut - m.d_cut)) / m.d_cut;
        const double t = 0.5 * (cos(M_PI * x) + 1.0), dt = -0.5 * M_PI * sin(M_PI * x) / m.d_cut;
        dv = dv * t + v * dt;
        v *= t;
    }
}

__global__ void __launch_bounds__(256)
k_bond_derivs(bop_model m, int n, long P, const int *__restrict__ species, const int *__restrict__ row_ptr,
              const int *__restrict__ nbr_j, const double *__restrict__ nbr_d, double *__restrict__ dH)
{
    using D3 = Dual<3>;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int i = pair_owner(row_ptr, n, p), j = nbr_j[p];
    D3 d[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        d[x] = dc<3>(nbr_d[3 * p + x]);
        d[x].d[x] = 1.0;
    }
    const D3 r = dsqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const D3 l = d[0] / r, mm = d[1] / r, nn = d[2] / r;
    const int si = species[i], sj = species[j];
    const bool ok = si >= 0 && si < m.n_species && sj >= 0 && sj < m.n_species;
    const int pr = ok ? si * m.n_species + sj : 0;
    D3 V[3];
    const int chans[3] = {BOP_DDS, BOP_DDP, BOP_DDD};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double v, dv;
        bond_integral_dr(m, pr, chans[c], r.v, v, dv);
        V[c] = dc<3>(v);
#pragma unroll
        for (int x = 0; x < 3; ++x) V[c].d[x] = dv * r.d[x];
    }
    // real d harmonics (order z2, zx, yz, x2-y2, xy) and their gradients in u
    const double s3 = 1.7320508075688772;
    D3 Y[5], G[5][3];
    Y[0] = nn * nn - 0.5 * (l * l + mm * mm);
    Y[1] = s3 * (l * nn);
    Y[2] = s3 * (mm * nn);
    Y[3] = (0.5 * s3) * (l * l - mm * mm);
    Y[4] = s3 * (l * mm);
    G[0][0] = -l;          G[0][1] = -mm;          G[0][2] = 2.0 * nn;
    G[1][0] = s3 * nn;     G[1][1] = dc<3>(0.0);   G[1][2] = s3 * l;
    G[2][0] = dc<3>(0.0);  G[2][1] = s3 * nn;      G[2][2] = s3 * mm;
    G[3][0] = s3 * l;      G[3][1] = -s3 * mm;     G[3][2] = dc<3>(0.0);
    G[4][0] = s3 * mm;     G[4][1] = s3 * l;       G[4][2] = dc<3>(0.0);
    double *out = dH + p * 3 * BOP_D_PACKED;
#pragma unroll
    for (int a = 0; a < 5; ++a)
#pragma unroll
        for (int b = a; b < 5; ++b) {
            const D3 ps = Y[a] * Y[b];
            const D3 gg = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
            const D3 pp = (1.0 / 3.0) * (gg - 4.0 * ps);
            const D3 pd = (a == b ? 1.0 : 0.0) - ps - pp;
            const D3 h = V[0] * ps + V[1] * pp + V[2] * pd;
#pragma unroll
            for (int x = 0; x < 3; ++x) out[x * BOP_D_PACKED + d_packed_index(a, b)] = ok ? h.d[x] : __builtin_nan("");
        }
#pragma unroll
    for (int x = 0; x < 3; ++x) out[x * BOP_D_PACKED + BOP_D_PACKED - 1] = 0.0;
}

// ---------------------------------------------------------------------------
// Theta~ passes
// ---------------------------------------------------------------------------
struct FBatch {
    int first, count;
};

// H and the derivative blocks are read at wave-uniform addresses through the
// constant address space, so that their loads stay scalar loads also where the
// kernel issues LDS-DMA loads (which the compiler takes as possible writes)
template <typename T> using CT = const __attribute__((address_space(4))) T;

// row offset of X^l in a tile's level store
struct LevelOffsets {
    long off[F_MAXN + 1];
};

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// X^0 = unit columns and G^n = w_n e_c on the seed rows; a failed tile (its
// support did not fit the plan) poisons its seeds' pair gradients with NaN.
template <typename T, int NO>
__global__ void k_finit(FBatch bt, int n, const double *__restrict__ w, const int *__restrict__ sizes_,
                        const char *tiles_base, size_t tile_stride, const int *__restrict__ row_ptr, T *xlev,
                        size_t xlev_rows, T *gbuf, size_t g_rows, double *gpair, double *theta_on)
{
    const int t = blockIdx.x;
    if (t >= bt.count) return;
    const int tile = bt.first + t;
    const int *sizes = sizes_ + tile * (MAXK + 2);
    const int *sup = (const int *)(tiles_base + tile_stride * tile);
    constexpr int SR = NO * 64;
    if (sizes[0] < 0) {
        for (int b = 0; b < sizes[1]; ++b) {
            const int g = sup[b];
            for (long p = row_ptr[g] + threadIdx.x; p < row_ptr[g + 1]; p += blockDim.x)
                for (int x = 0; x < 3; ++x) unsafeAtomicAdd(&gpair[3 * p + x], __builtin_nan(""));
            if (theta_on && threadIdx.x < NO) unsafeAtomicAdd(&theta_on[(long)g * NO + threadIdx.x], __builtin_nan(""));
        }
        return;
    }
    const int Bt = sizes[0];
    T *X0 = xlev + (size_t)t * xlev_rows * SR;
    T *Gn = gbuf + ((size_t)t * 2 + (n & 1)) * g_rows * SR;
    for (int e = threadIdx.x; e < Bt * SR; e += blockDim.x) {
        const int l = e / SR, rest = e % SR, a = rest / 64, c = rest % 64;
        const bool own = c == l * NO + a;
        X0[e] = own ? T(1) : T(0);
        Gn[e] = own ? (T)w[((long)sup[l] * NO + a) * (n + 1) + n] : T(0);
    }
}

// One forward (BWD = false: X^lev = H X^(lev-1)) or backward (BWD = true:
// G^lev = w_lev e_c + H G^(lev+1) with the Theta~ contraction against X^lev)
// pass over a batch of tiles.  Launch numbering as in the moment passes: all
// chunks of a tile on one XCD, rows dealt to the chunks in wave-sized groups.
// A row's neighbour slots go in groups of GS: the group's rows of the operand
// are gathered before any is used.  In the backward pass each lane's three
// contraction values per slot go to the wave's LDS block [3 GS][65] and are
// summed over the 64 columns by eight lanes per value, each adding every
// eighth column, then three exchanges among the eight (a shuffle tree per
// value, or a few lanes adding 32 columns each, cost more instructions).
constexpr int GS = 2;                         // slots per gather group
constexpr int TSTRIDE = 65;                   // LDS row of one value (64 columns + pad)

template <typename T, int NO, bool BWD>
__global__ void __launch_bounds__(FW)
k_fstep(FBatch bt, int lev, int n, int K, int nch, int chunk_rows, int deg_max, int rows_cap,
        const int *__restrict__ row_ptr, const double *__restrict__ H_on, const T *__restrict__ H,
        const double *__restrict__ dH, const double *__restrict__ w, const int *__restrict__ rev,
        const int *__restrict__ sizes_, const char *tiles_base, size_t tile_stride, T *xlev, size_t xlev_rows,
        LevelOffsets lo, T *gbuf, size_t g_rows, double *accb, double *gpair, double *aonb,
        double *theta_on)
{
    constexpr int NB = BOP_D_PACKED;
    constexpr int SR = NO * 64;
    __shared__ double s_t[BWD ? NWF : 1][BWD ? 3 * GS * TSTRIDE : 1];
    __shared__ unsigned s_sink[sizeof(T) == 4 ? NWF : 1][64];   // LDS copies of the L2 touches, never read
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int t = (q / nch) * 8 + xcd, chunk = q % nch;
    if (t >= bt.count) return;
    const int tile = bt.first + t;
    const int *sizes = sizes_ + tile * (MAXK + 2);
    if (sizes[0] < 0) return;
    const int Lc = min(min(lev, n - lev), K);
    const int Lp = BWD ? min(min(lev + 1, n - lev - 1), K) : min(min(lev - 1, n - lev + 1), K);
    const int nrow = sizes[Lc];
    const int nct = tile_chunks(nrow, chunk_rows, NWF);
    if (chunk >= nct) return;
    const int RS = nct * NWF;
    const int *sup = (const int *)(tiles_base + tile_stride * tile);
    const int *rinfo = sup + rows_cap;
    const int *lnb = rinfo + rows_cap;
    T *Xt = xlev + (size_t)t * xlev_rows * SR;
    T *Gt = gbuf + (size_t)t * 2 * g_rows * SR;
    const T *src = BWD ? Gt + (size_t)((lev + 1) & 1) * g_rows * SR : Xt + (size_t)lo.off[lev - 1] * SR;
    T *dst = BWD ? Gt + (size_t)(lev & 1) * g_rows * SR : Xt + (size_t)lo.off[lev] * SR;
    const T *Xk = Xt + (size_t)lo.off[BWD ? lev : 0] * SR;
    double *acc_t = accb + (size_t)t * rows_cap * deg_max * 3;
    double *aon_t = aonb + (size_t)t * rows_cap * NO;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double *st = &s_t[BWD ? wv : 0][0];
    const int Bt = sizes[0];
    T wl = T(0);                       // the lane's column weight w_lev
    if (BWD && lev >= 1 && lane < Bt * NO) wl = (T)w[((long)sup[lane / NO] * NO + lane % NO) * (n + 1) + lev];
    // reduction lanes: value vg of the group, columns sg, sg + 8, ..., sg + 56
    const int vg = lane >> 3, sg = lane & 7;
    // the next row's atom, layer word, slot list and first pair are fetched
    // while the current row computes
    int l = chunk * NWF + wv;
    int g_n = 0, info_n = 0, slots_n = 0, p0_n = 0;
    if (l < nrow) {
        g_n = __builtin_amdgcn_readfirstlane(sup[l]);
        info_n = __builtin_amdgcn_readfirstlane(rinfo[l]);
        slots_n = lane < deg_max ? lnb[(long)l * deg_max + lane] : 0;
        p0_n = __builtin_amdgcn_readfirstlane(row_ptr[g_n]);
    }
    for (; l < nrow; l += RS) {
        const int g = g_n, info = info_n, slots = slots_n, p0 = p0_n;
        if (l + RS < nrow) {
            g_n = __builtin_amdgcn_readfirstlane(sup[l + RS]);
            info_n = __builtin_amdgcn_readfirstlane(rinfo[l + RS]);
            slots_n = lane < deg_max ? lnb[(long)(l + RS) * deg_max + lane] : 0;
            p0_n = __builtin_amdgcn_readfirstlane(row_ptr[g_n]);
        }
        const int L = info & 255, n1 = (info >> 8) & 255, n2 = (info >> 16) & 255, n3 = (info >> 24) & 255;
        const int nval = Lp >= L + 1 ? n3 : (Lp == L ? n2 : n1);
        const int *lrow = lnb + (long)l * deg_max;
        const bool has_prev = L <= Lp;
        T acc[NO], xk[NO], xs[NO];
#pragma unroll
        for (int a = 0; a < NO; ++a) {
            xs[a] = has_prev ? src[(size_t)l * SR + a * 64 + lane] : T(0);
            acc[a] = (T)H_on[(long)g * NO + a] * xs[a];
            xk[a] = BWD ? Xk[(size_t)l * SR + a * 64 + lane] : T(0);
        }
        // a row's pair sums run from its first backward pass (lev = n - L, at
        // most n - 1) to its last (lev = L)
        const bool first = BWD && lev == min(n - L, n - 1), last = BWD && lev == L;
        double *acc_row = acc_t + (size_t)l * deg_max * 3;
        if (BWD && theta_on) {
            // onsite elements Theta~_(ia,ia): X^lev[i a] G^(lev+1)[i a] summed
            // over the columns, kept like the pair sums from the row's first
            // to its last pass; formed before the slots, so that the row's own
            // G^(lev+1) holds no registers across the slot loop
#pragma unroll
            for (int a = 0; a < NO; ++a) st[a * TSTRIDE + lane] = (double)xk[a] * (double)xs[a];
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_wave_barrier();
            double v = 0.0;
            if (vg < NO) {
                const double *row = st + vg * TSTRIDE + sg;
#pragma unroll
                for (int c = 0; c < 8; ++c) v += row[8 * c];
            }
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            if (sg == 0 && vg < NO) {
                double *ap = aon_t + (size_t)l * NO + vg;
                if (first && last) unsafeAtomicAdd(&theta_on[(long)g * NO + vg], v);
                else if (first) *ap = v;
                else if (last) unsafeAtomicAdd(&theta_on[(long)g * NO + vg], *ap + v);
                else *ap += v;
            }
            __builtin_amdgcn_wave_barrier();
        }
        for (int s0 = 0; s0 < nval; s0 += GS) {
            if (sizeof(T) == 4) {
                // FP32 vectors: the next group's H blocks (and derivative
                // blocks) are fetched into L2 by an LDS-DMA load whose LDS copy
                // is never read, so that their scalar loads find them there
                // (with FP64 vectors this costs the backward pass an occupancy
                // step and gains nothing)
                const int u = lane >> 2, part = lane & 3;
                const int sn = s0 + GS + u;
                const int sw = __shfl(slots, sn < 64 ? sn : 0);
                if (u < GS && sn < nval && (BWD || part == 0)) {
                    const long pn = (long)p0 + (sw & 255);
                    const void *a = part == 0 ? (const void *)(H + pn * NB) : (const void *)(dH + (pn * 3 + part - 1) * NB);
                    __builtin_amdgcn_global_load_lds(a, (__attribute__((address_space(3))) void *)&s_sink[wv][0], 4, 0, 0);
                }
            }
            T xn[GS][NO];
#pragma unroll
            for (int u = 0; u < GS; ++u) {
                const int su = s0 + u < nval ? s0 + u : s0;
                const int jl = __builtin_amdgcn_readlane(slots, su) >> 8;
#pragma unroll
                for (int b = 0; b < NO; ++b) xn[u][b] = src[(size_t)jl * SR + b * 64 + lane];
            }
            asm volatile("" ::: "memory");    // keep the group's gathers ahead of their uses
#pragma unroll
            for (int u = 0; u < GS; ++u) {
                if (s0 + u >= nval) break;
                const long pp = (long)p0 + (__builtin_amdgcn_readlane(slots, s0 + u) & 255);
                const CT<T> *h = (const CT<T> *)(H + pp * NB);
#pragma unroll
                for (int a = 0; a < NO; ++a)
#pragma unroll
                    for (int b = 0; b < NO; ++b) acc[a] = fma(h[d_packed_index(a, b)], xn[u][b], acc[a]);
                // the contraction of the pair's canonical direction only (the
                // one of lower index): g_reverse(p) = -g_p
                if (BWD && __builtin_amdgcn_readfirstlane(rev[pp]) > pp) {
                    const CT<double> *dh = (const CT<double> *)(dH + pp * 3 * NB);
                    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
                    for (int a = 0; a < NO; ++a)
#pragma unroll
                        for (int b = a; b < NO; ++b) {
                            const double sab = a == b ? (double)xk[a] * (double)xn[u][a]
                                                      : (double)xk[a] * (double)xn[u][b] + (double)xk[b] * (double)xn[u][a];
                            const int e = d_packed_index(a, b);
                            t0 = fma(sab, dh[e], t0);
                            t1 = fma(sab, dh[NB + e], t1);
                            t2 = fma(sab, dh[2 * NB + e], t2);
                        }
                    st[(3 * u) * TSTRIDE + lane] = t0;
                    st[(3 * u + 1) * TSTRIDE + lane] = t1;
                    st[(3 * u + 2) * TSTRIDE + lane] = t2;
                } else if (BWD) {
                    st[(3 * u) * TSTRIDE + lane] = 0.0;
                    st[(3 * u + 1) * TSTRIDE + lane] = 0.0;
                    st[(3 * u + 2) * TSTRIDE + lane] = 0.0;
                }
            }
            if (BWD) {
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_s_waitcnt(0xc07f);        // the group's LDS writes are done
                __builtin_amdgcn_wave_barrier();
                const int ng = 3 * min(GS, nval - s0);
                double v = 0.0;
                if (vg < ng) {
                    const double *row = st + vg * TSTRIDE + sg;
#pragma unroll
                    for (int c = 0; c < 8; ++c) v += row[8 * c];
                }
                v += __shfl_xor(v, 1);
                v += __shfl_xor(v, 2);
                v += __shfl_xor(v, 4);
                if (sg == 0 && vg < ng) {
                    const int s = s0 + vg / 3, x = vg % 3;
                    const long pp = (long)p0 + (lrow[s] & 255);
                    double *ap = acc_row + s * 3 + x;
                    if (rev[pp] > pp) {
                        if (first && last) unsafeAtomicAdd(&gpair[3 * pp + x], 2.0 * v);
                        else if (first) *ap = v;
                        else if (last) unsafeAtomicAdd(&gpair[3 * pp + x], 2.0 * (*ap + v));
                        else *ap += v;
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (BWD && first != last) {
            // slots whose operand is zero at this pass: start their sums at
            // zero (first pass) or hand them on (last pass)
            for (int e = lane; e < 3 * (n3 - nval); e += 64) {
                const int s = nval + e / 3, x = e % 3;
                const long pp = (long)p0 + (lrow[s] & 255);
                double *ap = acc_row + s * 3 + x;
                if (rev[pp] <= pp) continue;
                if (first) *ap = 0.0;
                else unsafeAtomicAdd(&gpair[3 * pp + x], 2.0 * *ap);
            }
        }
        if (BWD) {
            if (lev == 0) continue;          // G^0 is not needed
            if (L == 0) {
#pragma unroll
                for (int a = 0; a < NO; ++a)
                    if (lane == l * NO + a) acc[a] += wl;
            }
        }
#pragma unroll
        for (int a = 0; a < NO; ++a) __builtin_nontemporal_store(acc[a], &dst[(size_t)l * SR + a * 64 + lane]);
    }
}

// reverse pair of p = (i -> j, shift s): the pair (j -> i, -s); -1 if absent
__global__ void __launch_bounds__(256)
k_reverse(int n, long P, const int *__restrict__ row_ptr, const int *__restrict__ nbr_j,
          const int *__restrict__ nbr_shift, int *__restrict__ rev)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int i = pair_owner(row_ptr, n, p), j = nbr_j[p];
    const int s0 = nbr_shift[3 * p], s1 = nbr_shift[3 * p + 1], s2 = nbr_shift[3 * p + 2];
    int found = -1;
    for (int q = row_ptr[j]; q < row_ptr[j + 1]; ++q)
        if (nbr_j[q] == i && nbr_shift[3 * q] == -s0 && nbr_shift[3 * q + 1] == -s1 && nbr_shift[3 * q + 2] == -s2) {
            found = q;
            break;
        }
    rev[p] = found;
}

// F_k = sum over k's pairs p of g_p - g_rev(p), in pair order
__global__ void __launch_bounds__(256)
k_force_sum(int n, const int *__restrict__ row_ptr, const int *__restrict__ rev, const double *__restrict__ gpair,
            double *__restrict__ F)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    for (int p = row_ptr[k]; p < row_ptr[k + 1]; ++p) {
        const int q = rev[p];
        const double r0 = q >= 0 ? gpair[3L * q] : __builtin_nan("");
        const double r1 = q >= 0 ? gpair[3L * q + 1] : __builtin_nan("");
        const double r2 = q >= 0 ? gpair[3L * q + 2] : __builtin_nan("");
        f0 += gpair[3L * p] - r0;
        f1 += gpair[3L * p + 1] - r1;
        f2 += gpair[3L * p + 2] - r2;
    }
    F[3L * k] = f0;
    F[3L * k + 1] = f1;
    F[3L * k + 2] = f2;
}

__global__ void k_fill(double *p, long n, double v)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

// ---------------------------------------------------------------------------
// workspaces
// ---------------------------------------------------------------------------
struct WeightsWs {
    double *dN, *Drow, *part, *ebar;
    size_t bytes;
};

WeightsWs carve_weights(void *base, long R, int n_max)
{
    WeightsWs w{};
    char *p = (char *)base;
    auto take = [&](size_t b) { char *r = p; p += align_up(b, 256); return (void *)r; };
    w.dN = (double *)take(sizeof(double) * (size_t)R * (n_max + 1));
    w.Drow = (double *)take(sizeof(double) * (size_t)R);
    w.part = (double *)take(sizeof(double) * 2 * (size_t)((R + WT - 1) / WT + 1));
    w.ebar = (double *)take(sizeof(double));
    w.bytes = (size_t)(p - (char *)base);
    return w;
}

// rows of a tile's level store: X^l on layers <= min(l, n - l)
LevelOffsets level_offsets(const bop_plan &p, long *total)
{
    LevelOffsets lo{};
    const int n = p.n_max, K = n / 2;
    long o = 0;
    for (int l = 0; l < n; ++l) {
        lo.off[l] = o;
        const int h = std::min(std::min(l, n - l), K);
        o += p.rows_k[h];
    }
    lo.off[n] = o;
    *total = o;
    return lo;
}

struct ForcesWs {
    char *xlev, *gbuf;
    double *accb, *gpair, *aonb;
    int *rev;
    size_t xlev_rows, g_rows, bytes;
};

ForcesWs carve_forces(void *base, const bop_plan &p, long P, int bt)
{
    ForcesWs f{};
    char *c = (char *)base;
    auto take = [&](size_t b) { char *r = c; c += align_up(b, 256); return r; };
    long rows = 0;
    level_offsets(p, &rows);
    const size_t elem = p.dtype == BOP_F64 ? 8 : 4;
    const size_t row_bytes = elem * p.n_orb * 64;
    f.xlev_rows = (size_t)rows;
    f.g_rows = (size_t)p.rows_cap;
    f.gpair = (double *)take(sizeof(double) * 3 * (size_t)(P > 0 ? P : 1));
    f.rev = (int *)take(sizeof(int) * (size_t)(P > 0 ? P : 1));
    f.accb = (double *)take(sizeof(double) * 3 * (size_t)p.rows_cap * p.deg_max * bt);
    f.aonb = (double *)take(sizeof(double) * (size_t)p.rows_cap * p.n_orb * bt);
    f.xlev = take(row_bytes * f.xlev_rows * bt);
    f.gbuf = take(row_bytes * 2 * f.g_rows * bt);
    f.bytes = (size_t)(c - (char *)base);
    return f;
}

int default_force_batch(const bop_plan &p, long P)
{
    // tiles whose vectors are live at once: at most 24 GiB of them (a quarter
    // of the free memory if that is less), a multiple of 8, at least 8
    const size_t one = carve_forces(nullptr, p, P, 1).bytes - carve_forces(nullptr, p, P, 0).bytes;
    size_t budget = 24ull << 30, mem_free = 0, mem_total = 0;
    if (hipMemGetInfo(&mem_free, &mem_total) == hipSuccess && mem_free / 4 < budget) budget = mem_free / 4;
    long bt = one ? (long)(budget / one) : 8;
    bt = bt < 8 ? 8 : (bt / 8) * 8;
    if (bt > p.n_tiles) bt = p.n_tiles > 0 ? p.n_tiles : 1;
    return (int)bt;
}

template <typename T>
int run_forces(const bop_plan &p, const char *mws, const int *row_ptr, const double *H_on, const T *H,
               const double *dH, const double *w, const ForcesWs &f, int bt_max, double *theta_on, hipStream_t st)
{
    constexpr int NO = 5;
    const Layout lay = make_layout(p, map_workgroups(p.n_atoms, p.n_tiles));
    const int *sizes = (const int *)(mws + lay.sizes);
    const char *tiles = mws + lay.tiles;
    long rows = 0;
    const LevelOffsets lo = level_offsets(p, &rows);
    const int n = p.n_max, K = n / 2;
    T *xlev = (T *)f.xlev, *gbuf = (T *)f.gbuf;
    for (int first = 0; first < p.n_tiles; first += bt_max) {
        FBatch bt{first, std::min(bt_max, p.n_tiles - first)};
        k_finit<T, NO><<<bt.count, 256, 0, st>>>(bt, n, w, sizes, tiles, lay.tile_stride, row_ptr, xlev,
                                                 f.xlev_rows, gbuf, f.g_rows, f.gpair, theta_on);
        BOP_LAUNCHED();
        const int nb8 = (bt.count + 7) / 8;
        auto grid = [&](int lev) {
            const int h = std::min(std::min(lev, n - lev), K);
            const int nch = (p.rows_k[h] + F_CHUNK - 1) / F_CHUNK;
            return nch;
        };
        for (int l = 1; l < n; ++l) {
            const int nch = grid(l);
            k_fstep<T, NO, false><<<(unsigned)(nb8 * 8 * nch), FW, 0, st>>>(
                bt, l, n, K, nch, F_CHUNK, p.deg_max, p.rows_cap, row_ptr, H_on, H, dH, w, f.rev, sizes, tiles,
                lay.tile_stride, xlev, f.xlev_rows, lo, gbuf, f.g_rows, f.accb, f.gpair, f.aonb, nullptr);
            BOP_LAUNCHED();
        }
        for (int k = n - 1; k >= 0; --k) {
            const int nch = grid(k);
            k_fstep<T, NO, true><<<(unsigned)(nb8 * 8 * nch), FW, 0, st>>>(
                bt, k, n, K, nch, F_CHUNK, p.deg_max, p.rows_cap, row_ptr, H_on, H, dH, w, f.rev, sizes, tiles,
                lay.tile_stride, xlev, f.xlev_rows, lo, gbuf, f.g_rows, f.accb, f.gpair, f.aonb, theta_on);
            BOP_LAUNCHED();
        }
    }
    return BOP_OK;
}

}  // namespace
}  // namespace bop

using namespace bop;

extern "C" size_t bop_weights_workspace_size(int n_rows, int n_max)
{
    if (n_rows < 0 || n_max < 1 || n_max > F_MAXN) return 0;
    return carve_weights(nullptr, n_rows, n_max).bytes + 256;
}

extern "C" int bop_weights(int n_rows, int n_max, int n_exp, const double *mu, const double *H_on,
                           const double *E_F, double *w, void *ws, size_t ws_bytes, hipStream_t stream)
{
    BOP_REQUIRE(n_rows >= 0, BOP_E_ARG, "bop_weights: n_rows < 0");
    BOP_REQUIRE(n_max >= 1 && n_max <= F_MAXN, BOP_E_UNSUPPORTED, "bop_weights: n_max must be 1..%d", F_MAXN);
    BOP_REQUIRE(n_exp >= 1 && n_exp <= 1024, BOP_E_UNSUPPORTED, "bop_weights: n_exp must be 1..1024");
    if (n_rows == 0) return BOP_OK;
    BOP_REQUIRE(mu && H_on && E_F && w, BOP_E_ARG, "bop_weights: NULL array");
    WeightsWs ww = carve_weights(ws, n_rows, n_max);
    BOP_REQUIRE(ws && ws_bytes >= ww.bytes, BOP_E_CAPACITY, "bop_weights: workspace of %zu bytes needed", ww.bytes);
    const long nt = (long)n_rows * n_max;
    const unsigned g = (unsigned)((nt + WT - 1) / WT);
    // chain depth L = max(#a, #b) = (n_max + 1) / 2 levels below the delay level
    if ((n_max + 1) / 2 <= 9)
        k_weights<9><<<g, WT, 0, stream>>>(n_rows, n_max, n_exp, mu, H_on, E_F, w, ww.dN, ww.Drow);
    else
        k_weights<11><<<g, WT, 0, stream>>>(n_rows, n_max, n_exp, mu, H_on, E_F, w, ww.dN, ww.Drow);
    BOP_LAUNCHED();
    const unsigned rb = (unsigned)((n_rows + WT - 1) / WT);
    k_ebar_part<<<rb, WT, 0, stream>>>(n_rows, H_on, ww.Drow, ww.part);
    k_ebar<<<1, WT, 0, stream>>>(rb, ww.part, ww.ebar);
    BOP_LAUNCHED();
    const long ne = (long)n_rows * (n_max + 1);
    k_wfinish<<<(unsigned)((ne + WT - 1) / WT), WT, 0, stream>>>(ne, n_max + 1, w, ww.dN, E_F, ww.ebar, w);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" int bop_bond_derivatives(const bop_model *model, int n, const int *species, const int *row_ptr,
                                    const int *nbr_j, const double *nbr_d, long P, double *dH, hipStream_t stream)
{
    BOP_REQUIRE(model && n >= 0 && P >= 0, BOP_E_ARG, "bop_bond_derivatives: bad arguments");
    BOP_REQUIRE(model->n_orb == 5, BOP_E_UNSUPPORTED, "bop_bond_derivatives: d band (n_orb 5) only");
    BOP_REQUIRE(model->n_species >= 1 && model->n_species <= BOP_MAX_SPECIES, BOP_E_UNSUPPORTED,
                "bop_bond_derivatives: 1..%d species supported", BOP_MAX_SPECIES);
    if (P == 0) return BOP_OK;
    BOP_REQUIRE(species && row_ptr && nbr_j && nbr_d && dH, BOP_E_ARG, "bop_bond_derivatives: NULL array");
    k_bond_derivs<<<(unsigned)((P + 255) / 256), 256, 0, stream>>>(*model, n, P, species, row_ptr, nbr_j, nbr_d, dH);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" size_t bop_forces_workspace_size(const bop_plan *plan, long n_pairs, int batch_tiles)
{
    if (!plan || n_pairs < 0 || plan->n_max < 1 || plan->n_max > F_MAXN) return 0;
    const int bt = batch_tiles > 0 ? std::min(batch_tiles, std::max(plan->n_tiles, 1))
                                   : default_force_batch(*plan, n_pairs);
    return carve_forces(nullptr, *plan, n_pairs, bt).bytes + 256;
}

extern "C" int bop_forces(const bop_plan *plan, const void *moments_ws, const int *row_ptr, const int *nbr_j,
                          const int *nbr_shift, long n_pairs, const double *H_on, const void *H_bond,
                          const double *dH, const double *w, int batch_tiles, double *F, double *theta_on,
                          void *ws, size_t ws_bytes, hipStream_t stream)
{
    BOP_REQUIRE(plan && n_pairs >= 0, BOP_E_ARG, "bop_forces: bad arguments");
    BOP_REQUIRE(plan->n_orb == 5, BOP_E_UNSUPPORTED, "bop_forces: d band (n_orb 5) only");
    BOP_REQUIRE(plan->dtype == BOP_F64 || plan->dtype == BOP_F32, BOP_E_UNSUPPORTED,
                "bop_forces: vectors in FP64 or FP32 only");
    BOP_REQUIRE(plan->n_max >= 1 && plan->n_max <= F_MAXN, BOP_E_UNSUPPORTED, "bop_forces: n_max must be 1..%d",
                F_MAXN);
    BOP_REQUIRE(plan->r_max == 0.0, BOP_E_UNSUPPORTED, "bop_forces: no path radius");
    const int n = plan->n_atoms;
    if (n == 0) return BOP_OK;
    BOP_REQUIRE(moments_ws && row_ptr && nbr_j && nbr_shift && H_on && H_bond && dH && w && F, BOP_E_ARG,
                "bop_forces: NULL array");
    const int bt = batch_tiles > 0 ? std::min(batch_tiles, std::max(plan->n_tiles, 1))
                                   : default_force_batch(*plan, n_pairs);
    ForcesWs f = carve_forces(ws, *plan, n_pairs, bt);
    BOP_REQUIRE(ws && ws_bytes >= f.bytes, BOP_E_CAPACITY, "bop_forces: workspace of %zu bytes needed, %zu given",
                f.bytes, ws_bytes);
    const long ng = 3 * n_pairs;
    if (ng > 0) k_fill<<<(unsigned)((ng + 255) / 256), 256, 0, stream>>>(f.gpair, ng, 0.0);
    if (theta_on)
        k_fill<<<(unsigned)(((long)n * 5 + 255) / 256), 256, 0, stream>>>(theta_on, (long)n * 5, 0.0);
    if (n_pairs > 0)
        k_reverse<<<(unsigned)((n_pairs + 255) / 256), 256, 0, stream>>>(n, n_pairs, row_ptr, nbr_j, nbr_shift,
                                                                         f.rev);
    BOP_LAUNCHED();
    const int rc = plan->dtype == BOP_F64
                       ? run_forces<double>(*plan, (const char *)moments_ws, row_ptr, H_on, (const double *)H_bond,
                                            dH, w, f, bt, theta_on, stream)
                       : run_forces<float>(*plan, (const char *)moments_ws, row_ptr, H_on, (const float *)H_bond, dH,
                                           w, f, bt, theta_on, stream);
    if (rc != BOP_OK) return rc;
    k_force_sum<<<(unsigned)((n + 255) / 256), 256, 0, stream>>>(n, row_ptr, f.rev, f.gpair, F);
    BOP_LAUNCHED();
    return BOP_OK;
}

// Eq. BOP_SCF summed over an atom's orbitals (one onsite shift per atom):
// Delta_i = sum_a Theta~_(ia,ia) - N_i = dU/d(shift_i)
__global__ void __launch_bounds__(256)
k_scf_target(int n, int no, const double *__restrict__ theta_on, const double *__restrict__ N_atom,
             double *__restrict__ delta)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int a = 0; a < no; ++a) s += theta_on[(long)i * no + a];
    delta[i] = s - N_atom[i];
}

extern "C" int bop_scf_target(int n_atoms, int n_orb, const double *theta_on, const double *N_atom, double *delta,
                              hipStream_t stream)
{
    BOP_REQUIRE(n_atoms >= 0 && n_orb >= 1, BOP_E_ARG, "bop_scf_target: bad arguments");
    if (n_atoms == 0) return BOP_OK;
    BOP_REQUIRE(theta_on && N_atom && delta, BOP_E_ARG, "bop_scf_target: NULL array");
    k_scf_target<<<(unsigned)((n_atoms + 255) / 256), 256, 0, stream>>>(n_atoms, n_orb, theta_on, N_atom, delta);
    BOP_LAUNCHED();
    return BOP_OK;
}
