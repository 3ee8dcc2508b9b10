// Tile plan and workspace layout shared by the moment passes and the force
// passes: per-tile support sizes, the tile records (support rows, layer and
// slot counts, neighbour slots, row masks) written by the prepare pass, and
// where the X buffers, chunk partials and Lanczos coefficients live in a
// bop_moments workspace.
#pragma once
#include "bop_internal.h"

namespace bop {

constexpr int MAX_NMAX = 40;
constexpr int MAXK = MAX_NMAX / 2;
constexpr int HDR = 256;            // header ints: [0] queue, [1] error, [2] max rows, [3] max degree,
                                    // [8 + k] max rows of U^k (plan)
constexpr int LC_N = 8;             // Lanczos column coefficients per lane and tile

// Row assignment of the step kernels: a tile with nrow rows at this step uses
// nct = tile_chunks(..) of the launch's chunks, and chunk c < nct takes the
// wave-sized row groups c, c + nct, c + 2 nct, ...  nct depends on the tile
// alone, so the grouping of the partial sums (and the rounding of the moments)
// does not change with the other tiles of the plan.
__device__ inline int tile_chunks(int nrow, int chunk_rows, int nw)
{
    return min((nrow + chunk_rows - 1) / chunk_rows, (nrow + nw - 1) / nw);
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
// Bytes of one row of X (all 64 columns): n_orb values per column in
// FP64/FP32 ([n_orb][64] per row), or n_orb padded to the MFMA slot width in
// BF16 ([64][slot width] per row).
__host__ __device__ inline size_t x_row_bytes(int dtype, int n_orb)
{
    if (dtype == BOP_BF16) return 2ull * 64 * (n_orb <= 8 ? 8 : 16);
    return (dtype == BOP_F64 ? 8ull : (dtype == BOP_F16 ? 2ull : 4ull)) * n_orb * 64;
}

struct Layout {
    size_t sizes;       // int [n_tiles][MAXK + 2]: rows of U^k per tile; [0] = -1 marks a failed tile
    size_t tiles;       // per tile: sup[rows_cap], rinfo[rows_cap], lnb[rows_cap * deg_max], rmask[rows_cap]
    size_t tile_stride;
    size_t x;           // X buffers: batch x 2 x rows_cap x n_orb x 64 (also prepare's maps)
    size_t x_stride;    // bytes of one X buffer
    size_t part;        // double [batch][chunks][2][64]
    size_t lc;          // double [batch][LC_N][64]: Lanczos column coefficients
    size_t bytes;
};

// Where each step's chunk partials start (doubles, for batch_tiles tiles) and
// how many chunks the step has.
struct StepParts {
    long off[MAXK + 2];
    int nch[MAXK + 2];
    size_t total_chunks;
};

__host__ __device__ inline StepParts step_parts(const bop_plan &p)
{
    StepParts sp{};
    const int K = p.n_max / 2, steps = K + (p.n_max & 1);
    size_t tot = 0;
    for (int k = 1; k <= steps && k <= MAXK + 1; ++k) {
        const int rows_k = k > K ? p.rows_k[K] : p.rows_k[k];
        sp.nch[k] = (rows_k + p.chunk_rows - 1) / p.chunk_rows;
        sp.off[k] = (long)(tot * 2 * 64 * (size_t)p.batch_tiles);
        tot += (size_t)sp.nch[k];
    }
    sp.total_chunks = tot;
    return sp;
}

__host__ __device__ inline Layout make_layout(const bop_plan &p, int n_prep_wg)
{
    Layout L;
    size_t o = HDR;
    auto take = [&](size_t b) { size_t r = o; o += (b + 255) / 256 * 256; return r; };
    L.sizes = take(4ull * p.n_tiles * (MAXK + 2));
    L.tile_stride = (4ull * p.rows_cap * (3 + p.deg_max) + 255) / 256 * 256;   // sup, rinfo, lnb, row masks
    L.tiles = take(L.tile_stride * p.n_tiles);
    L.x_stride = (x_row_bytes(p.dtype, p.n_orb) * p.rows_cap + 255) / 256 * 256;
    size_t xb = L.x_stride * (p.batch_tiles >= 2 ? 2 * (size_t)p.batch_tiles : 4);
    size_t maps = (size_t)n_prep_wg * ((4ull * p.n_atoms + 255) / 256 * 256);
    L.x = take(xb > maps ? xb : maps);
    // chunk partials: one step's worth for the Lanczos form (three per chunk at
    // its last level), every step's for the moment form (two per chunk,
    // reduced after the batch's last step)
    const size_t nch = (p.rows_cap + p.chunk_rows - 1) / p.chunk_rows;
    const size_t nch_all = step_parts(p).total_chunks;
    L.part = take(8ull * 64 * (3 * nch > 2 * nch_all ? 3 * nch : 2 * nch_all) * p.batch_tiles);
    L.lc = take(8ull * LC_N * 64 * p.batch_tiles);
    L.bytes = o;
    return L;
}

// Workgroups of the plan and prepare passes: two per CU, but at most about
// 1 GiB of per-workgroup global->local maps.
inline int map_workgroups(int n_atoms, int n_tiles)
{
    size_t per = align_up(4ull * n_atoms, 256) * 2;
    long cap = (long)((1ull << 30) / (per ? per : 1));
    long w = 2L * device_cus();
    if (w > cap) w = cap;
    if (w > n_tiles) w = n_tiles;
    return w < 1 ? 1 : (int)w;
}

}  // namespace bop
