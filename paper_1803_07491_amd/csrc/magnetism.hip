// Collinear magnetism (arXiv:1803.07491, Sec. II "Hamiltonian": the two spin
// channels are computed one after the other, each like a non-magnetic
// calculation; App. A.2.2, collinear onsite levels; App. A.1 Eq. TB-UX).
//
// The channels share the bond blocks and differ in their onsite levels,
//   E_iav = H0_ia + shift_i - (-1)^v B_z + (1/2) (-1)^v I_i m_i,
// with (-1)^v = -1 for the up channel (the majority channel of a positive
// moment is lowered by I m / 2).  Both channels' rows are stacked, up atoms
// then down atoms, in every per-row and per-atom buffer, so that the H.X
// passes run once per channel on the same plan and the FP64 tail runs once
// over the stacked rows.  The energy call counts both spins of a row (factor
// 2); the Fermi level of the stacked rows for 2 N_e electrons is therefore the
// level at which the channels together hold N_e, and its per-atom outputs are
// halved afterwards to give per-channel values.
#include "bop_internal.h"

namespace bop {
namespace {

constexpr int MT = 256;

__global__ void k_spin_shifts(int n, const int *__restrict__ species, bop_magnetism mag,
                              const double *__restrict__ shift, const double *__restrict__ moment,
                              double *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sp = species[i];
    // a species outside the table gives NaN levels, never an index past it
    const double I = (sp >= 0 && sp < BOP_MAX_SPECIES) ? mag.stoner[sp] : __builtin_nan("");
    const double s = shift ? shift[i] : 0.0, m = moment ? moment[i] : 0.0;
    out[i] = s + mag.B_z - 0.5 * I * m;
    out[n + i] = s - mag.B_z + 0.5 * I * m;
}

// halve the stacked per-atom outputs (per channel now), m_i = N_iup - N_idown,
// per-block partials of I_i m_i^2
__global__ void __launch_bounds__(MT)
k_mag_post(int n, const int *__restrict__ species, bop_magnetism mag, double *__restrict__ N_atom,
           double *__restrict__ U_atom, double *__restrict__ dos_atom, double *__restrict__ m_out,
           double *__restrict__ part)
{
    __shared__ double s_red[MT / 64];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double x = 0.0;
    if (i < n) {
        const double nu = 0.5 * N_atom[i], nd = 0.5 * N_atom[n + i];
        N_atom[i] = nu;
        N_atom[n + i] = nd;
        U_atom[i] *= 0.5;
        U_atom[n + i] *= 0.5;
        dos_atom[i] *= 0.5;
        dos_atom[n + i] *= 0.5;
        const double m = nu - nd;
        m_out[i] = m;
        const int sp = species[i];
        x = ((sp >= 0 && sp < BOP_MAX_SPECIES) ? mag.stoner[sp] : __builtin_nan("")) * m * m;
    }
    x = block_combine(x, 0, s_red);
    if (threadIdx.x == 0) part[blockIdx.x] = x;
}

__global__ void __launch_bounds__(MT)
k_mag_totals(unsigned nblk, const double *__restrict__ part, double *__restrict__ U_total, double *__restrict__ U_X)
{
    __shared__ double s_comb[MT / 64];
    const double t = partials_combine(part, nblk, 1, 0, 0, s_comb);
    if (threadIdx.x == 0) {
        U_X[0] = -0.25 * t;
        U_total[0] *= 0.5;
    }
}

// q_i, m_out - m_i, the new shift before the mean is removed, and per-block
// max |q|, max |dm|, sum of new shifts
__global__ void __launch_bounds__(MT)
k_mag_measure(int n, const double *__restrict__ N_sp, const double *__restrict__ dos_sp,
              const double *__restrict__ n0, const double *__restrict__ m_out, const double *__restrict__ moment,
              const double *__restrict__ shift, double mix, double n_floor, double *__restrict__ q,
              double *__restrict__ part)
{
    __shared__ double s_a[MT / 64], s_b[MT / 64], s_c[MT / 64];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double mq = 0.0, mm = 0.0, sum = 0.0;
    if (i < n) {
        const double qi = N_sp[i] + N_sp[n + i] - n0[i];
        q[i] = qi;
        mq = fabs(qi);
        mm = fabs(m_out[i] - moment[i]);
        const double d = dos_sp[i] + dos_sp[n + i];
        sum = shift[i] + mix * qi / (d > n_floor ? d : n_floor);
    }
    for (int o = 32; o > 0; o >>= 1) {
        mq = fmax(mq, __shfl_xor(mq, o));
        mm = fmax(mm, __shfl_xor(mm, o));
        sum += __shfl_xor(sum, o);
    }
    if ((threadIdx.x & 63) == 0) {
        s_a[threadIdx.x >> 6] = mq;
        s_b[threadIdx.x >> 6] = mm;
        s_c[threadIdx.x >> 6] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int w = 0; w < MT / 64; ++w) {
            a = fmax(a, s_a[w]);
            b = fmax(b, s_b[w]);
            c += s_c[w];
        }
        part[3 * blockIdx.x] = a;
        part[3 * blockIdx.x + 1] = b;
        part[3 * blockIdx.x + 2] = c;
    }
}

__global__ void __launch_bounds__(MT)
k_mag_total(unsigned nblk, int n, double tol, double tol_m, const double *__restrict__ part,
            double *__restrict__ max_d, int *__restrict__ converged, double *__restrict__ mean)
{
    __shared__ double s_comb[MT / 64];
    const double a = fmax(0.0, partials_combine(part, nblk, 3, 0, 2, s_comb));
    const double b = fmax(0.0, partials_combine(part, nblk, 3, 1, 2, s_comb));
    const double c = partials_combine(part, nblk, 3, 2, 0, s_comb);
    if (threadIdx.x == 0) {
        max_d[0] = a;
        max_d[1] = b;
        converged[0] = a < tol && b < tol_m;
        mean[0] = c / n;
    }
}

__global__ void k_mag_apply(int n, const double *__restrict__ q, const double *__restrict__ dos_sp,
                            const double *__restrict__ m_out, double mix, double mix_m, double n_floor,
                            const int *__restrict__ converged, const double *__restrict__ mean,
                            double *__restrict__ shift, double *__restrict__ moment)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || converged[0]) return;
    const double d = dos_sp[i] + dos_sp[n + i];
    shift[i] = (shift[i] + mix * q[i] / (d > n_floor ? d : n_floor)) - mean[0];
    moment[i] = moment[i] + mix_m * (m_out[i] - moment[i]);
}

}  // namespace
}  // namespace bop

using namespace bop;

extern "C" int bop_spin_shifts(int n_atoms, const int *species, const bop_magnetism *mag, const double *shift,
                               const double *moment, double *shift_spin, hipStream_t stream)
{
    BOP_REQUIRE(n_atoms >= 0 && mag, BOP_E_ARG, "bop_spin_shifts: bad arguments");
    if (n_atoms == 0) return BOP_OK;
    BOP_REQUIRE(species && shift_spin, BOP_E_ARG, "bop_spin_shifts: NULL array");
    k_spin_shifts<<<(n_atoms + MT - 1) / MT, MT, 0, stream>>>(n_atoms, species, *mag, shift, moment, shift_spin);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" int bop_mag_energy(const bop_system *sys, const bop_magnetism *mag, const double *shift,
                              const double *moment, double *m_out, double *U_X, hipStream_t stream)
{
    BOP_REQUIRE(sys && mag && m_out && U_X, BOP_E_ARG, "bop_mag_energy: NULL argument");
    const int n = sys->n_atoms, no = sys->model.n_orb;
    BOP_REQUIRE(n > 0 && sys->species, BOP_E_ARG, "bop_mag_energy: empty system");
    BOP_REQUIRE(sys->method == 0 || sys->method == 1, BOP_E_ARG, "bop_mag_energy: method must be 0 or 1");
    for (int s = 0; s < sys->model.n_species; ++s)
        BOP_REQUIRE(std::isfinite(mag->stoner[s]), BOP_E_ARG, "bop_mag_energy: Stoner parameter not finite");
    const long R = (long)n * no;
    const int na = sys->n_max >= 1 ? (sys->n_max - 1) / 2 + 1 : 0, nb = sys->n_max / 2;
    // the channel shifts go through N_atom, which bop_energy overwrites later
    double *sh = sys->N_atom;
    int rc = bop_spin_shifts(n, sys->species, mag, shift, moment, sh, stream);
    if (rc) return rc;
    for (int c = 0; c < 2; ++c) {
        double *H_on = sys->H_on + c * R;
        rc = bop_build_H(&sys->model, n, sys->species, sh + (size_t)c * n, sys->row_ptr, sys->nbr_j, nullptr,
                         sys->n_pairs, sys->dtype, H_on, nullptr, stream);
        if (rc) return rc;
        if (sys->method == 0)
            rc = bop_moments(&sys->plan, sys->row_ptr, H_on, sys->H_bond, sys->mu + c * R * (sys->n_max + 1),
                             sys->moments_ws, sys->moments_ws_bytes, stream);
        else
            rc = bop_lanczos(&sys->plan, sys->row_ptr, H_on, sys->H_bond, sys->a + c * R * na,
                             sys->b + c * R * (nb + 1), sys->flags + c * R, sys->moments_ws, sys->moments_ws_bytes,
                             stream);
        if (rc) return rc;
    }
    const double *mu = sys->method == 0 ? sys->mu : nullptr;
    rc = bop_recursion((int)(2 * R), sys->n_max, mu, 0, 0.0, 0.0, sys->a, sys->b, sys->a_inf, sys->b_inf,
                       sys->flags, stream);
    if (rc) return rc;
    rc = bop_energy(2 * n, no, sys->n_max, sys->n_exp, mu, sys->a, sys->b, sys->a_inf, sys->b_inf, sys->H_on,
                    2.0 * sys->n_elec, 0, sys->E_F, sys->N_atom, sys->U_atom, sys->dos_atom, sys->U_total,
                    sys->flags, sys->energy_ws, sys->energy_ws_bytes, stream);
    if (rc) return rc;
    double *part = energy_ws_scratch(sys->energy_ws, 2 * R, sys->n_exp);
    const unsigned nblk = (unsigned)((n + MT - 1) / MT);
    k_mag_post<<<nblk, MT, 0, stream>>>(n, sys->species, *mag, sys->N_atom, sys->U_atom, sys->dos_atom, m_out,
                                        part);
    k_mag_totals<<<1, MT, 0, stream>>>(nblk, part, sys->U_total, U_X);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" int bop_mag_scf_step(const bop_system *sys, const bop_magnetism *mag, double mix, double mix_m,
                                double n_floor, double tol, double tol_m, double *shift, double *moment,
                                double *m_out, double *q, double *U_X, double *max_d, int *converged,
                                hipStream_t stream)
{
    BOP_REQUIRE(sys && mag && shift && moment && m_out && q && U_X && max_d && converged && sys->n0, BOP_E_ARG,
                "bop_mag_scf_step: NULL argument");
    int rc = bop_mag_energy(sys, mag, shift, moment, m_out, U_X, stream);
    if (rc) return rc;
    const int n = sys->n_atoms, no = sys->model.n_orb;
    double *part = energy_ws_scratch(sys->energy_ws, 2L * n * no, sys->n_exp);
    const unsigned nblk = (unsigned)((n + MT - 1) / MT);
    double *mean = part + 3 * (size_t)nblk;
    k_mag_measure<<<nblk, MT, 0, stream>>>(n, sys->N_atom, sys->dos_atom, sys->n0, m_out, moment, shift, mix,
                                           n_floor, q, part);
    k_mag_total<<<1, MT, 0, stream>>>(nblk, n, tol, tol_m, part, max_d, converged, mean);
    BOP_LAUNCHED();
    k_mag_apply<<<nblk, MT, 0, stream>>>(n, q, sys->dos_atom, m_out, mix, mix_m, n_floor, converged, mean, shift,
                                         moment);
    BOP_LAUNCHED();
    return BOP_OK;
}
