// One local-charge-neutrality self-consistency step (App. A.3 Eq. BOP_LCN of
// arXiv:1803.07491, with the linear input/output mixing of Sec. II
// "Self-consistency").  The onsite levels are rebuilt from the per-atom
// shifts, the energy path is re-run, and the shifts are updated on the device:
//   q_i = N_i - n0_i;  converged if max |q_i| < tol (shifts unchanged), else
//   shift_i += mix q_i / max(n_i(E_F), n_floor), then the mean shift is
//   removed (shifting every level and E_F together leaves the state unchanged).
// Both global reductions use per-block partials summed in a fixed order.
#include "bop_internal.h"

namespace bop {
namespace {

constexpr int ST = 256;

__global__ void __launch_bounds__(ST)
k_scf_measure(int n, const double *__restrict__ N_atom, const double *__restrict__ dos,
              const double *__restrict__ n0, const double *__restrict__ shift, double mix, double n_floor,
              double *__restrict__ q, double *__restrict__ part)
{
    __shared__ double s_m[ST / 64], s_s[ST / 64];
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double mq = 0.0, sum = 0.0;
    if (i < n) {
        double qi = N_atom[i] - n0[i];
        q[i] = qi;
        mq = fabs(qi);
        double den = dos[i] > n_floor ? dos[i] : n_floor;
        sum = shift[i] + mix * qi / den;
    }
    for (int o = 32; o > 0; o >>= 1) { mq = fmax(mq, __shfl_xor(mq, o)); sum += __shfl_xor(sum, o); }
    if ((threadIdx.x & 63) == 0) { s_m[threadIdx.x >> 6] = mq; s_s[threadIdx.x >> 6] = sum; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0, t = 0.0;
        for (int w = 0; w < ST / 64; ++w) { m = fmax(m, s_m[w]); t += s_s[w]; }
        part[2 * blockIdx.x] = m;
        part[2 * blockIdx.x + 1] = t;
    }
}

// max |q| and the mean new shift from the block partials (one block, fixed
// order; a launch of its own, so that no block needs a device-scope fence)
__global__ void __launch_bounds__(ST)
k_scf_total(unsigned n_blocks, int n, double tol, const double *__restrict__ part, double *__restrict__ max_dq,
            int *__restrict__ converged, double *__restrict__ mean_out)
{
    __shared__ double s_comb[ST / 64];
    const double m = fmax(0.0, partials_combine(part, n_blocks, 2, 0, 2, s_comb));
    const double t = partials_combine(part, n_blocks, 2, 1, 0, s_comb);
    if (threadIdx.x == 0) {
        max_dq[0] = m;
        converged[0] = m < tol;
        mean_out[0] = t / n;
    }
}

__global__ void k_scf_apply(int n, const double *__restrict__ q, const double *__restrict__ dos,
                            double mix, double n_floor, const int *__restrict__ converged,
                            const double *__restrict__ mean, double *__restrict__ shift)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || converged[0]) return;
    double den = dos[i] > n_floor ? dos[i] : n_floor;
    shift[i] = (shift[i] + mix * q[i] / den) - mean[0];
}

}  // namespace
}  // namespace bop

using namespace bop;

extern "C" int bop_scf_step(const bop_system *sys, double mix, double n_floor, double tol, double *shift,
                            double *q, double *max_dq, int *converged, hipStream_t stream)
{
    BOP_REQUIRE(sys && shift && q && max_dq && converged, BOP_E_ARG, "bop_scf_step: NULL argument");
    const int n = sys->n_atoms, no = sys->model.n_orb;
    BOP_REQUIRE(n > 0 && sys->n0 && sys->species, BOP_E_ARG, "bop_scf_step: empty system");
    int rc = bop_build_H(&sys->model, n, sys->species, shift, sys->row_ptr, sys->nbr_j, nullptr,
                         sys->n_pairs, sys->dtype, sys->H_on, nullptr, stream);
    if (rc) return rc;
    BOP_REQUIRE(sys->method == 0 || sys->method == 1, BOP_E_ARG, "bop_scf_step: method must be 0 or 1");
    const double *mu = sys->method == 0 ? sys->mu : nullptr;
    if (sys->method == 0)
        rc = bop_moments(&sys->plan, sys->row_ptr, sys->H_on, sys->H_bond, sys->mu, sys->moments_ws,
                         sys->moments_ws_bytes, stream);
    else
        rc = bop_lanczos(&sys->plan, sys->row_ptr, sys->H_on, sys->H_bond, sys->a, sys->b, sys->flags,
                         sys->moments_ws, sys->moments_ws_bytes, stream);
    if (rc) return rc;
    rc = bop_recursion(n * no, sys->n_max, mu, 0, 0.0, 0.0, sys->a, sys->b, sys->a_inf, sys->b_inf,
                       sys->flags, stream);
    if (rc) return rc;
    rc = bop_energy(n, no, sys->n_max, sys->n_exp, mu, sys->a, sys->b, sys->a_inf, sys->b_inf,
                    sys->H_on, sys->n_elec, 0, sys->E_F, sys->N_atom, sys->U_atom, sys->dos_atom,
                    sys->U_total, sys->flags, sys->energy_ws, sys->energy_ws_bytes, stream);
    if (rc) return rc;
    double *part = energy_ws_scratch(sys->energy_ws, (long)n * no, sys->n_exp);
    const unsigned nb = (unsigned)((n + ST - 1) / ST);
    double *mean = part + 2 * (size_t)nb;    // one slot past the partials
    k_scf_measure<<<nb, ST, 0, stream>>>(n, sys->N_atom, sys->dos_atom, sys->n0, shift, mix, n_floor, q, part);
    k_scf_total<<<1, ST, 0, stream>>>(nb, n, tol, part, max_dq, converged, mean);
    BOP_LAUNCHED();
    k_scf_apply<<<nb, ST, 0, stream>>>(n, q, sys->dos_atom, mix, n_floor, converged, mean, shift);
    BOP_LAUNCHED();
    return BOP_OK;
}
