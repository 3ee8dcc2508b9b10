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

// ---------------------------------------------------------------------------
// Broyden mixing (Sec. II "Self-consistency", mixer (ii); Broyden's second
// method, the update of the inverse Jacobian).  Residual F_i = q_i /
// max(n_i(E_F), n_floor) (the linear mixer's output step); H_0 = -mix I;
// with s = x_n - x_(n-1), y = F_n - F_(n-1):
//   u = (s - H_(n-1) y) / (y.y),  H_n = H_(n-1) + u y^T,  x_(n+1) = x_n - H_n F_n,
// H kept as -mix I + sum_k u_k y_k^T; every hist + 1 steps the history starts
// again from H_0.  Dot products: per-block partials, then one block per dot
// summing them in block order (deterministic).
// ---------------------------------------------------------------------------
constexpr int MAX_HIST = 64;

struct BroydenWs {
    double *x_prev, *F_prev, *F, *U, *Y, *coef, *part;
    int nblk;
    size_t bytes;
};

BroydenWs broyden_carve(void *base, int n, int hist)
{
    BroydenWs w{};
    char *p = (char *)base;
    auto take = [&](size_t b) { char *r = p; p += align_up(b, 256); return (double *)r; };
    const size_t v = sizeof(double) * (size_t)n;
    w.nblk = (n + ST - 1) / ST;
    w.x_prev = take(v);
    w.F_prev = take(v);
    w.F = take(v);
    w.U = take(v * (size_t)hist);
    w.Y = take(v * (size_t)hist);
    w.coef = take(sizeof(double) * 2 * (MAX_HIST + 2));
    w.part = take(sizeof(double) * (size_t)w.nblk * (MAX_HIST + 2));
    w.bytes = (size_t)(p - (char *)base);
    return w;
}

// q_i, F_i and per-block max |q_i|
__global__ void __launch_bounds__(ST)
k_bro_residual(int n, const double *__restrict__ N_atom, const double *__restrict__ dos,
               const double *__restrict__ n0, double n_floor, double *__restrict__ q, double *__restrict__ F,
               double *__restrict__ part)
{
    __shared__ double s_m[ST / 64];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double mq = 0.0;
    if (i < n) {
        const double qi = N_atom[i] - n0[i];
        q[i] = qi;
        mq = fabs(qi);
        F[i] = qi / (dos[i] > n_floor ? dos[i] : n_floor);
    }
    for (int o = 32; o > 0; o >>= 1) mq = fmax(mq, __shfl_xor(mq, o));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = mq;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < ST / 64; ++w) m = fmax(m, s_m[w]);
        part[blockIdx.x] = m;
    }
}

__global__ void __launch_bounds__(ST)
k_bro_maxq(unsigned nblk, double tol, const double *__restrict__ part, double *__restrict__ max_dq,
           int *__restrict__ converged)
{
    __shared__ double s_comb[ST / 64];
    const double m = fmax(0.0, partials_combine(part, nblk, 1, 0, 2, s_comb));
    if (threadIdx.x == 0) {
        max_dq[0] = m;
        converged[0] = m < tol;
    }
}

// y = F - F_prev into Y[j-1], s = x - x_prev into U[j-1]
__global__ void k_bro_sy(int n, int j, const int *__restrict__ converged, const double *__restrict__ x,
                         const double *__restrict__ x_prev, const double *__restrict__ F,
                         const double *__restrict__ F_prev, double *__restrict__ U, double *__restrict__ Y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || converged[0]) return;
    Y[(size_t)(j - 1) * n + i] = F[i] - F_prev[i];
    U[(size_t)(j - 1) * n + i] = x[i] - x_prev[i];
}

// partials of V[d] . w for d < nd (block b, dot d)
__global__ void __launch_bounds__(ST)
k_bro_dots(int n, int nd, const int *__restrict__ converged, const double *__restrict__ V,
           const double *__restrict__ w, double *__restrict__ part)
{
    __shared__ double s_red[ST / 64];
    if (converged[0]) return;
    const int d = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v = i < n ? V[(size_t)d * n + i] * w[i] : 0.0;
    v = block_combine(v, 0, s_red);
    if (threadIdx.x == 0) part[(size_t)d * gridDim.x + blockIdx.x] = v;
}

__global__ void __launch_bounds__(ST)
k_bro_dots_sum(unsigned nblk, const int *__restrict__ converged, const double *__restrict__ part,
               double *__restrict__ out)
{
    __shared__ double s_comb[ST / 64];
    if (converged[0]) return;
    const int d = blockIdx.x;
    const double t = partials_combine(part + (size_t)d * nblk, nblk, 1, 0, 0, s_comb);
    if (threadIdx.x == 0) out[d] = t;
}

// U[j-1] = (s + mix y - sum_(d < j-1) U[d] c_d) / (y.y), with c = coef[0..j-2],
// y.y = coef[j-1]; a zero update when y.y = 0
__global__ void k_bro_u(int n, int j, double mix, const int *__restrict__ converged, const double *__restrict__ coef,
                        double *__restrict__ U, const double *__restrict__ Y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || converged[0]) return;
    const double yy = coef[j - 1];
    const size_t o = (size_t)(j - 1) * n + i;
    double v = U[o] + mix * Y[o];
    for (int d = 0; d < j - 1; ++d) v -= U[(size_t)d * n + i] * coef[d];
    U[o] = yy > 0.0 ? v / yy : 0.0;
}

// x_new = x + mix F - sum_(d < j) U[d] e_d, e = coef2; x_prev = x, F_prev = F;
// per-block sums of x_new for the mean
__global__ void __launch_bounds__(ST)
k_bro_apply(int n, int j, double mix, const int *__restrict__ converged, const double *__restrict__ e,
            const double *__restrict__ U, const double *__restrict__ F, double *__restrict__ x,
            double *__restrict__ x_prev, double *__restrict__ F_prev, double *__restrict__ part)
{
    __shared__ double s_red[ST / 64];
    if (converged[0]) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double xn = 0.0;
    if (i < n) {
        const double xi = x[i], fi = F[i];
        xn = xi + mix * fi;
        for (int d = 0; d < j; ++d) xn -= U[(size_t)d * n + i] * e[d];
        x_prev[i] = xi;
        F_prev[i] = fi;
        x[i] = xn;
    }
    xn = block_combine(xn, 0, s_red);
    if (threadIdx.x == 0) part[blockIdx.x] = xn;
}

__global__ void __launch_bounds__(ST)
k_bro_mean(unsigned nblk, int n, const int *__restrict__ converged, const double *__restrict__ part,
           double *__restrict__ mean)
{
    __shared__ double s_comb[ST / 64];
    if (converged[0]) return;
    const double t = partials_combine(part, nblk, 1, 0, 0, s_comb);
    if (threadIdx.x == 0) mean[0] = t / n;
}

__global__ void k_bro_gauge(int n, const int *__restrict__ converged, const double *__restrict__ mean,
                            double *__restrict__ x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || converged[0]) return;
    x[i] -= mean[0];
}

}  // namespace
}  // namespace bop

using namespace bop;

static int scf_energy(const bop_system *sys, const double *shift, hipStream_t stream);

extern "C" size_t bop_broyden_workspace_size(int n_atoms, int hist)
{
    if (n_atoms <= 0 || hist < 0 || hist > MAX_HIST) return 0;
    return broyden_carve(nullptr, n_atoms, hist).bytes + 256;
}

extern "C" int bop_scf_step_broyden(const bop_system *sys, double mix, double n_floor, double tol, int iter,
                                    int hist, double *shift, double *q, double *max_dq, int *converged, void *ws,
                                    size_t ws_bytes, hipStream_t stream)
{
    BOP_REQUIRE(sys && shift && q && max_dq && converged, BOP_E_ARG, "bop_scf_step_broyden: NULL argument");
    const int n = sys->n_atoms;
    BOP_REQUIRE(n > 0 && sys->n0 && sys->species, BOP_E_ARG, "bop_scf_step_broyden: empty system");
    BOP_REQUIRE(iter >= 0 && hist >= 0 && hist <= MAX_HIST, BOP_E_ARG,
                "bop_scf_step_broyden: iter >= 0 and 0 <= hist <= %d required", MAX_HIST);
    BroydenWs w = broyden_carve(ws, n, hist);
    BOP_REQUIRE(ws && ws_bytes >= w.bytes, BOP_E_CAPACITY, "bop_scf_step_broyden: workspace of %zu bytes needed",
                w.bytes);
    int rc = scf_energy(sys, shift, stream);
    if (rc) return rc;
    const unsigned nb = (unsigned)w.nblk;
    k_bro_residual<<<nb, ST, 0, stream>>>(n, sys->N_atom, sys->dos_atom, sys->n0, n_floor, q, w.F, w.part);
    k_bro_maxq<<<1, ST, 0, stream>>>(nb, tol, w.part, max_dq, converged);
    BOP_LAUNCHED();
    // position in the history: j = 0 starts again from H_0 (linear mixing)
    const int j = iter % (hist + 1);
    double *c = w.coef, *e = w.coef + (MAX_HIST + 2);
    if (j >= 1) {
        k_bro_sy<<<nb, ST, 0, stream>>>(n, j, converged, shift, w.x_prev, w.F, w.F_prev, w.U, w.Y);
        // c_d = Y[d] . y for d < j - 1 and y . y (d = j - 1)
        k_bro_dots<<<dim3(nb, (unsigned)j), ST, 0, stream>>>(n, j, converged, w.Y, w.Y + (size_t)(j - 1) * n,
                                                            w.part);
        k_bro_dots_sum<<<(unsigned)j, ST, 0, stream>>>(nb, converged, w.part, c);
        k_bro_u<<<nb, ST, 0, stream>>>(n, j, mix, converged, c, w.U, w.Y);
        // e_d = Y[d] . F for d < j
        k_bro_dots<<<dim3(nb, (unsigned)j), ST, 0, stream>>>(n, j, converged, w.Y, w.F, w.part);
        k_bro_dots_sum<<<(unsigned)j, ST, 0, stream>>>(nb, converged, w.part, e);
        BOP_LAUNCHED();
    }
    k_bro_apply<<<nb, ST, 0, stream>>>(n, j, mix, converged, e, w.U, w.F, shift, w.x_prev, w.F_prev, w.part);
    k_bro_mean<<<1, ST, 0, stream>>>(nb, n, converged, w.part, c + MAX_HIST + 1);
    k_bro_gauge<<<nb, ST, 0, stream>>>(n, converged, c + MAX_HIST + 1, shift);
    BOP_LAUNCHED();
    return BOP_OK;
}

// The energy path at the current shifts: onsite levels, H.X passes,
// recursion, expansion, Fermi level and per-atom N, U and n(E_F).
static int scf_energy(const bop_system *sys, const double *shift, hipStream_t stream)
{
    const int n = sys->n_atoms, no = sys->model.n_orb;
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
    return bop_energy(n, no, sys->n_max, sys->n_exp, mu, sys->a, sys->b, sys->a_inf, sys->b_inf,
                      sys->H_on, sys->n_elec, 0, sys->E_F, sys->N_atom, sys->U_atom, sys->dos_atom,
                      sys->U_total, sys->flags, sys->energy_ws, sys->energy_ws_bytes, stream);
}

extern "C" int bop_scf_step(const bop_system *sys, double mix, double n_floor, double tol, double *shift,
                            double *q, double *max_dq, int *converged, hipStream_t stream)
{
    BOP_REQUIRE(sys && shift && q && max_dq && converged, BOP_E_ARG, "bop_scf_step: NULL argument");
    const int n = sys->n_atoms, no = sys->model.n_orb;
    BOP_REQUIRE(n > 0 && sys->n0 && sys->species, BOP_E_ARG, "bop_scf_step: empty system");
    int rc = scf_energy(sys, shift, stream);
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
