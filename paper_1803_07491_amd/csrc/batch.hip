// Batched form: many independent periodic structures as one block-diagonal
// neighbour graph, so that a single moment plan, prepare pass and moment
// launch sequence serves the whole batch.  This file only joins the
// per-structure neighbour lists (local atom indices) into global ones.
#include "bop_internal.h"

namespace bop {
namespace {

constexpr int CT = 256;

// structure of atom i (atom_off sorted, atom_off[0] = 0)
__device__ inline int struct_of(int i, const int *__restrict__ off, int n_structs)
{
    int lo = 0, hi = n_structs;        // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(CT)
k_concat_rows(int n_structs, int n, const int *__restrict__ atom_off, const int *__restrict__ pair_off,
              const int *__restrict__ row_ptr_local, const int *__restrict__ order_local, int *__restrict__ row_ptr,
              int *__restrict__ order)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == n) { row_ptr[n] = pair_off[n_structs]; return; }
    const int s = struct_of(i, atom_off, n_structs);
    const int li = i - atom_off[s];
    // structure s's local row_ptr (n_s + 1 entries) starts at atom_off[s] + s
    row_ptr[i] = pair_off[s] + row_ptr_local[atom_off[s] + s + li];
    order[i] = atom_off[s] + order_local[i];
}

__global__ void __launch_bounds__(CT)
k_concat_pairs(int n_structs, int n, const int *__restrict__ atom_off, const int *__restrict__ row_ptr,
               const int *__restrict__ nbr_j_local, int *__restrict__ nbr_j)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = struct_of(i, atom_off, n_structs);
    const int a = atom_off[s];
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) nbr_j[p] = a + nbr_j_local[p];
}

}  // namespace
}  // namespace bop

using namespace bop;

extern "C" int bop_batch_concat(int n_structs, int n_atoms, const int *atom_off, const int *pair_off,
                                const int *row_ptr_local, const int *nbr_j_local, const int *order_local,
                                int *row_ptr, int *nbr_j, int *order, hipStream_t stream)
{
    BOP_REQUIRE(n_structs >= 1 && n_atoms >= 0, BOP_E_ARG, "bop_batch_concat: bad sizes");
    BOP_REQUIRE(atom_off && pair_off && row_ptr_local && row_ptr && order && order_local, BOP_E_ARG,
                "bop_batch_concat: NULL array");
    const unsigned g1 = (unsigned)((n_atoms + 1 + CT - 1) / CT);
    k_concat_rows<<<g1, CT, 0, stream>>>(n_structs, n_atoms, atom_off, pair_off, row_ptr_local, order_local, row_ptr,
                                        order);
    BOP_LAUNCHED();
    if (n_atoms > 0) {
        BOP_REQUIRE(nbr_j_local && nbr_j, BOP_E_ARG, "bop_batch_concat: NULL pair array");
        k_concat_pairs<<<(unsigned)((n_atoms + CT - 1) / CT), CT, 0, stream>>>(n_structs, n_atoms, atom_off,
                                                                              row_ptr, nbr_j_local, nbr_j);
        BOP_LAUNCHED();
    }
    return BOP_OK;
}

extern "C" int bop_moments_batched(const bop_plan *plan, int n_structs, const int *atom_off, const int *pair_off,
                                   const int *row_ptr_local, const int *nbr_j_local, const int *order_local,
                                   int *row_ptr, int *nbr_j, int *order, const double *H_on, const void *H_bond,
                                   double *mu, void *ws, size_t ws_bytes, hipStream_t stream)
{
    BOP_REQUIRE(plan, BOP_E_ARG, "bop_moments_batched: plan is NULL");
    BOP_REQUIRE(plan->r_max == 0.0, BOP_E_UNSUPPORTED, "bop_moments_batched: no path radius");
    int rc = bop_batch_concat(n_structs, plan->n_atoms, atom_off, pair_off, row_ptr_local, nbr_j_local, order_local,
                              row_ptr, nbr_j, order, stream);
    if (rc != BOP_OK) return rc;
    rc = bop_moments_prepare(plan, row_ptr, nbr_j, order, nullptr, ws, ws_bytes, stream);
    if (rc != BOP_OK) return rc;
    return bop_moments(plan, row_ptr, H_on, H_bond, mu, ws, ws_bytes, stream);
}
