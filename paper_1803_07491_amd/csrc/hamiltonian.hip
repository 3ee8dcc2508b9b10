// Two-centre tight-binding Hamiltonian blocks (App. A.2.1 of arXiv:1803.07491:
// bond-frame block Eq. (Hij), bond integrals with the cosine taper
// Eq. (cutoff), rotation to the global frame Eq. (Hij_rot) with the matrices of
// App. D).
//
// One thread per directed pair p = (i -> j).  The bond frame has z' along the
// pair vector d; the block is R^T H^(b) R where R[a][b] is App. D's matrix with
// a the bond-frame orbital and b the global one (theta = polar angle of d,
// phi = its azimuth), evaluated from the direction cosines without
// trigonometric calls.  The model (a few kB) travels as a kernel argument.
#include "bop_internal.h"

#include <cmath>

namespace bop {
namespace {

__device__ inline double bond_integral(const bop_model &m, int pair, int ch, double r)
{
    double b0 = m.beta0[pair][ch];
    if (b0 == 0.0) return 0.0;
    double v = (m.form[pair][ch] == BOP_FORM_POWER) ? b0 * pow(m.r0[pair][ch] / r, m.q[pair][ch])
                                                    : b0 * exp(-m.q[pair][ch] * (r - m.r0[pair][ch]));
    if (m.d_cut > 0.0 && r >= m.r_cut - m.d_cut) {
        double x = (r - (m.r_cut - m.d_cut)) / m.d_cut;
        v *= 0.5 * (cos(M_PI * x) + 1.0);
    }
    return v;
}

template <typename T> __device__ inline T to_dtype(double v);
template <> __device__ inline double to_dtype<double>(double v) { return v; }
template <> __device__ inline float to_dtype<float>(double v) { return (float)v; }
template <> __device__ inline __hip_bfloat16 to_dtype<__hip_bfloat16>(double v) { return __float2bfloat16((float)v); }

// App. D, d block: rows = bond-frame orbital, columns = global orbital.
__device__ inline void rot_d(double ct, double st, double cp, double sp, double R[5][5])
{
    const double s3 = 1.7320508075688772, s34 = 0.8660254037844386;
    double c2t = ct * ct, s2t = st * st, c2p = cp * cp, s2p = sp * sp, cdp = c2p - s2p;
    R[0][0] = c2t - 0.5 * s2t;       R[0][1] = s3 * cp * st * ct;  R[0][2] = s3 * sp * st * ct;
    R[0][3] = cdp * s34 * s2t;       R[0][4] = s3 * sp * cp * s2t;
    R[1][0] = -s3 * st * ct;         R[1][1] = cp * (c2t - s2t);   R[1][2] = sp * (c2t - s2t);
    R[1][3] = cdp * st * ct;         R[1][4] = 2.0 * sp * cp * st * ct;
    R[2][0] = 0.0;                   R[2][1] = -sp * ct;           R[2][2] = cp * ct;
    R[2][3] = -2.0 * sp * cp * st;   R[2][4] = cdp * st;
    R[3][0] = s34 * s2t;             R[3][1] = -cp * st * ct;      R[3][2] = -sp * st * ct;
    R[3][3] = cdp * (c2t + 0.5 * s2t); R[3][4] = sp * cp * (c2t + 1.0);
    R[4][0] = 0.0;                   R[4][1] = sp * st;            R[4][2] = -cp * st;
    R[4][3] = -2.0 * sp * cp * ct;   R[4][4] = cdp * ct;
}

// App. D, p block (order p_z, p_x, p_y).
__device__ inline void rot_p(double ct, double st, double cp, double sp, double R[3][3])
{
    R[0][0] = ct;   R[0][1] = cp * st;  R[0][2] = sp * st;
    R[1][0] = -st;  R[1][1] = cp * ct;  R[1][2] = sp * ct;
    R[2][0] = 0.0;  R[2][1] = -sp;      R[2][2] = cp;
}

__device__ inline int owner_row(const int *__restrict__ row_ptr, int n, long p)
{
    int lo = 0, hi = n - 1;            // largest i with row_ptr[i] <= p
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (row_ptr[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_bonds_d(bop_model m, int n, long P, const int *__restrict__ species, const int *__restrict__ row_ptr,
          const int *__restrict__ nbr_j, const double *__restrict__ nbr_d, T *__restrict__ H, int ld)
{
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    int i = owner_row(row_ptr, n, p), j = nbr_j[p];
    double dx = nbr_d[3 * p], dy = nbr_d[3 * p + 1], dz = nbr_d[3 * p + 2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double l = dx / r, mm = dy / r, nn = dz / r;
    double st = sqrt(l * l + mm * mm), ct = nn, cp = 1.0, sp = 0.0;
    if (st > 0.0) { cp = l / st; sp = mm / st; }
    // a species outside the model gives NaN blocks (never an index past its tables)
    const int si = species[i], sj = species[j];
    const bool ok = si >= 0 && si < m.n_species && sj >= 0 && sj < m.n_species;
    int pr = ok ? si * m.n_species + sj : 0;
    double D[5] = { bond_integral(m, pr, BOP_DDS, r), bond_integral(m, pr, BOP_DDP, r),
                    bond_integral(m, pr, BOP_DDP, r), bond_integral(m, pr, BOP_DDD, r),
                    bond_integral(m, pr, BOP_DDD, r) };
    if (!ok)
        for (int c = 0; c < 5; ++c) D[c] = __builtin_nan("");
    double R[5][5];
    rot_d(ct, st, cp, sp, R);
    if constexpr (sizeof(T) >= 4) {
        // FP64/FP32: the symmetric block packed, upper triangle row-major
        T *out = H + p * BOP_D_PACKED;
#pragma unroll
        for (int b = 0; b < 5; ++b)
#pragma unroll
            for (int c = b; c < 5; ++c) {
                double s = 0.0;
#pragma unroll
                for (int a = 0; a < 5; ++a) s += R[a][b] * D[a] * R[a][c];
                out[d_packed_index(b, c)] = to_dtype<T>(s);
            }
        out[BOP_D_PACKED - 1] = to_dtype<T>(0.0);
        return;
    }
    T *out = H + p * 5 * ld;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 5; ++a) s += R[a][b] * D[a] * R[a][c];
            out[b * ld + c] = to_dtype<T>(s);
        }
        for (int c = 5; c < ld; ++c) out[b * ld + c] = to_dtype<T>(0.0);
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_bonds_spd(bop_model m, int n, long P, const int *__restrict__ species, const int *__restrict__ row_ptr,
            const int *__restrict__ nbr_j, const double *__restrict__ nbr_d, T *__restrict__ H, int ld)
{
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    int i = owner_row(row_ptr, n, p), j = nbr_j[p];
    double dx = nbr_d[3 * p], dy = nbr_d[3 * p + 1], dz = nbr_d[3 * p + 2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double l = dx / r, mm = dy / r, nn = dz / r;
    double st = sqrt(l * l + mm * mm), ct = nn, cp = 1.0, sp = 0.0;
    if (st > 0.0) { cp = l / st; sp = mm / st; }
    const int si = species[i], sj = species[j];
    const bool ok = si >= 0 && si < m.n_species && sj >= 0 && sj < m.n_species;
    int pr = ok ? si * m.n_species + sj : 0;
    double v[BOP_N_CHANNELS];
#pragma unroll
    for (int c = 0; c < BOP_N_CHANNELS; ++c) v[c] = ok ? bond_integral(m, pr, c, r) : __builtin_nan("");
    // block-diagonal rotation (1, R_p, R_d) as a full 9x9
    double Rp[3][3], Rd[5][5], R[9][9];
    rot_p(ct, st, cp, sp, Rp);
    rot_d(ct, st, cp, sp, Rd);
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
        for (int b = 0; b < 9; ++b) R[a][b] = 0.0;
    R[0][0] = 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) R[1 + a][1 + b] = Rp[a][b];
#pragma unroll
    for (int a = 0; a < 5; ++a)
#pragma unroll
        for (int b = 0; b < 5; ++b) R[4 + a][4 + b] = Rd[a][b];
    // bond-frame block of Eq. (Hij): entries (row, col, channel)
    constexpr int NE = 19;
    const int er[NE] = { 0, 0, 0, 1, 1, 1, 2, 2, 3, 3, 4, 4, 4, 5, 5, 6, 6, 7, 8 };
    const int ec[NE] = { 0, 1, 4, 0, 1, 4, 2, 5, 3, 6, 0, 1, 4, 2, 5, 3, 6, 7, 8 };
    const int ech[NE] = { BOP_SSS, BOP_SPS, BOP_SDS, BOP_PSS, BOP_PPS, BOP_PDS, BOP_PPP, BOP_PDP,
                          BOP_PPP, BOP_PDP, BOP_DSS, BOP_DPS, BOP_DDS, BOP_DPP, BOP_DDP, BOP_DPP,
                          BOP_DDP, BOP_DDD, BOP_DDD };
    // H[b][c] = sum_(a, a') R[a][b] Hb[a][a'] R[a'][c]
    T *out = H + p * 9 * ld;
#pragma unroll
    for (int b = 0; b < 9; ++b) {
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < NE; ++e) s += R[er[e]][b] * v[ech[e]] * R[ec[e]][c];
            out[b * ld + c] = to_dtype<T>(s);
        }
        for (int c = 9; c < ld; ++c) out[b * ld + c] = to_dtype<T>(0.0);
    }
}

__global__ void k_onsite(bop_model m, int n, const int *__restrict__ species, const double *__restrict__ shift,
                         double *__restrict__ H_on)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = species[i], no = m.n_orb;
    const bool ok = s >= 0 && s < m.n_species;
    double sh = shift ? shift[i] : 0.0;
    for (int a = 0; a < no; ++a) {
        int lq = (no == 5) ? 2 : (a == 0 ? 0 : (a < 4 ? 1 : 2));
        H_on[(long)i * no + a] = ok ? m.onsite[s][lq] + sh : __builtin_nan("");
    }
}

}  // namespace
}  // namespace bop

using namespace bop;
static_assert(sizeof(bop_model) <= 4000, "model must fit in the kernel argument segment");

extern "C" int bop_build_H(const bop_model *model, int n, const int *species, const double *shift,
                           const int *row_ptr, const int *nbr_j, const double *nbr_d, long P,
                           int dtype, double *H_on, void *H_bond, hipStream_t stream)
{
    BOP_REQUIRE(model && n >= 0 && P >= 0, BOP_E_ARG, "bop_build_H: bad arguments");
    BOP_REQUIRE(model->n_orb == 5 || model->n_orb == 9, BOP_E_UNSUPPORTED,
                "bop_build_H: n_orb must be 5 or 9 (got %d)", model->n_orb);
    BOP_REQUIRE(model->n_species >= 1 && model->n_species <= BOP_MAX_SPECIES, BOP_E_UNSUPPORTED,
                "bop_build_H: 1..%d species supported", BOP_MAX_SPECIES);
    if (dtype == BOP_F16) dtype = BOP_F32;     // FP16 storage of the vectors uses FP32 blocks
    BOP_REQUIRE(dtype == BOP_F64 || dtype == BOP_F32 || dtype == BOP_BF16, BOP_E_UNSUPPORTED,
                "bop_build_H: unknown dtype %d", dtype);
    BOP_REQUIRE(n == 0 || (species && H_on), BOP_E_ARG, "bop_build_H: species/H_on NULL");
    const int T = 256;
    if (n > 0) {
        k_onsite<<<(n + T - 1) / T, T, 0, stream>>>(*model, n, species, shift, H_on);
        BOP_LAUNCHED();
    }
    if (!H_bond || P == 0) return BOP_OK;
    BOP_REQUIRE(row_ptr && nbr_j && nbr_d, BOP_E_ARG, "bop_build_H: neighbour arrays NULL");
    unsigned g = (unsigned)((P + T - 1) / T);
    const int no = model->n_orb;
    const int ld = (dtype == BOP_BF16) ? (no <= 8 ? 8 : 16) : no;   // BF16: MFMA slot width
    if (no == 5) {
        if (dtype == BOP_F64) k_bonds_d<double><<<g, T, 0, stream>>>(*model, n, P, species, row_ptr, nbr_j, nbr_d, (double *)H_bond, ld);
        else if (dtype == BOP_F32) k_bonds_d<float><<<g, T, 0, stream>>>(*model, n, P, species, row_ptr, nbr_j, nbr_d, (float *)H_bond, ld);
        else k_bonds_d<__hip_bfloat16><<<g, T, 0, stream>>>(*model, n, P, species, row_ptr, nbr_j, nbr_d, (__hip_bfloat16 *)H_bond, ld);
    } else {
        if (dtype == BOP_F64) k_bonds_spd<double><<<g, T, 0, stream>>>(*model, n, P, species, row_ptr, nbr_j, nbr_d, (double *)H_bond, ld);
        else if (dtype == BOP_F32) k_bonds_spd<float><<<g, T, 0, stream>>>(*model, n, P, species, row_ptr, nbr_j, nbr_d, (float *)H_bond, ld);
        else k_bonds_spd<__hip_bfloat16><<<g, T, 0, stream>>>(*model, n, P, species, row_ptr, nbr_j, nbr_d, (__hip_bfloat16 *)H_bond, ld);
    }
    BOP_LAUNCHED();
    return BOP_OK;
}
