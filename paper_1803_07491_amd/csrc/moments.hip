// Orbital moments mu_ia^(n) = <i a|H^n|i a> (App. B.3 of arXiv:1803.07491,
// Eq. momDOS), computed from interference paths built iteratively,
// X^k = H X^(k-1) (Eq. xi_rec), and merged at the middle of each path
// (Eqs. xi_invert, xi_merge):
//     mu_2k = <X^k, X^k>,  mu_2k-1 = <X^(k-1), X^k>,  mu_2K+1 = <X^K, H X^K>.
//
// GPU design (not the paper's CPU scheme):
//  * A tile is a group of B spatially adjacent atoms; the B * n_orb unit start
//    vectors are the columns of X, one column per lane of a 64-wide wavefront.
//  * Each tile's K-hop support is found once per neighbour list (prepare pass)
//    by a deterministic breadth-first search, one workgroup per tile.  Up to
//    524,288 atoms, two bitmaps in LDS (visited atoms, atoms of the layer being
//    built) give each layer, listed in ascending atom index by a scan of the
//    layer bitmap; for larger structures every frontier (row, slot) claims its
//    neighbour with an atomic minimum on a per-workgroup global->local map and
//    the owners are compacted in (row, slot) order.  Either way local rows come
//    out in layer order independent of scheduling.  Each local row keeps its
//    neighbour slots sorted by the neighbour's layer: at step k the neighbours
//    whose X^(k-1) is non-zero form a prefix of that list.
//  * The steps are step-synchronous launches over a batch of tiles; a
//    wavefront owns a row and all 64 columns.  The row's H blocks reach the
//    wave's LDS slice by an asynchronous copy issued after the previous row
//    (FP32), or are read with scalar loads (FP64); neighbour rows of X^(k-1)
//    are coalesced vector loads in double-buffered groups; X^k is written with
//    non-temporal stores.  Blocks are numbered so that all chunks of a tile run
//    on one XCD (block b runs on XCD b mod 8) one tile after another, and the
//    rows are dealt to the tile's chunks in wave-sized groups round robin, so
//    the rows in flight on an XCD form one window of consecutive rows in layer
//    order.  Their neighbours then sit in a few nearby patches of adjacent
//    layers, and the ~15-fold reuse of every gathered row stays in the XCD's
//    L2 instead of going to memory.
//  * The plan pass only needs the layer sizes and finds them with one visited
//    bitmap in LDS (unordered appends).
//  * The moment dot products are fused into the step; per-chunk partial sums
//    (FP64) of every step are kept and reduced in chunk order after a batch's
//    last step, so results are deterministic for a given plan.
#include "bop_internal.h"
#include "tiles.h"

namespace bop {
namespace {

constexpr int UNSEEN = 0x7fffffff;
constexpr int CLAIM = 1 << 30;
constexpr int PLAN_T = 512;

// The global->local maps of the support search are private to one workgroup
// (all of whose waves share a CU), so workgroup scope is enough for them; it
// keeps the map traffic in the XCD's L2, where device-scope atomics and stores
// would go through to memory, the L2s of the XCDs not being coherent.
__device__ inline int wg_load(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ inline void wg_store(int *p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ inline void wg_min(int *p, int v)
{
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Maximum path radius: an atom belongs to a tile's support only if it lies
// within r_max of one of the tile's atoms, and a column keeps only the rows
// within r_max of its own atom.  Distances are minimum-image distances from
// the positions: fractional offsets rounded to the nearest integer, which is
// exact for offsets shorter than half the smallest cell height (the plan
// requires r_max below that).
struct Radius {
    int on;
    double r2;
    double A[9], Ai[9];          // cell rows a1, a2, a3 and the inverse
    const double *pos;
};

__device__ inline bool within(const Radius &R, const double *pj, const double *pt)
{
    const double d0 = pj[0] - pt[0], d1 = pj[1] - pt[1], d2 = pj[2] - pt[2];
    double f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f[a] = d0 * R.Ai[a] + d1 * R.Ai[3 + a] + d2 * R.Ai[6 + a];
        f[a] -= rint(f[a]);
    }
    double q = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double v = f[0] * R.A[c] + f[1] * R.A[3 + c] + f[2] * R.A[6 + c];
        q += v * v;
    }
    return q <= R.r2;
}

// whether atom j lies within r_max of any of the tile's Bt atoms (positions in tp)
__device__ inline bool inside_any(const Radius &R, int j, const double *tp, int Bt)
{
    if (!R.on) return true;
    const double pj[3] = {R.pos[3 * (long)j], R.pos[3 * (long)j + 1], R.pos[3 * (long)j + 2]};
    for (int t = 0; t < Bt; ++t)
        if (within(R, pj, tp + 3 * t)) return true;
    return false;
}

// the tile atoms' positions into LDS (tp: 3 doubles per atom, at most 64 atoms)
__device__ inline void tile_positions(const Radius &R, const int *sup, int Bt, double *tp)
{
    if (R.on)
        for (int e = threadIdx.x; e < 3 * Bt; e += blockDim.x) tp[e] = R.pos[3 * (long)sup[e / 3] + e % 3];
}

// exclusive prefix of a 0/1 flag over the workgroup; returns the position and
// writes the workgroup total
template <int WGT>
__device__ inline int wg_scan01(int own, int *s_wave, int &total)
{
    constexpr int NW = WGT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long b = __ballot(own);
    int pre = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) s_wave[w] = __popcll(b);
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        int c = s_wave[q];
        off += (q < w) ? c : 0;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return off + pre;
}

// Breadth-first k-hop support of one tile.  On return s_size[k] = |support of
// X^k| for k = 0..K (layer order), sup[0..s_size[K]) lists the global atoms and
// g2l maps them to local rows.  Returns -1 (with g2l restored) if the support
// would exceed rows_cap.
//
// Layer k: every (frontier row t, slot s) entry e = (t - begin) * deg_max + s,
// one per thread, proposes itself for its neighbour with an atomic minimum, and
// the neighbours won by their smallest entry are appended in entry order, so
// the row order does not depend on scheduling.
template <int WGT>
__device__ int bfs_tile(int tile, int B, int n_atoms, int K, const int *__restrict__ order,
                        const int *__restrict__ row_ptr, const int *__restrict__ nbr_j, int deg_max,
                        int *g2l, int *sup, int rows_cap, int *s_size, int *s_wave, int *s_flag,
                        const Radius &rad, double *s_tp)
{
    const int tid = threadIdx.x;
    const int first = tile * B;
    const int Bt = min(B, n_atoms - first);
    if (tid < Bt && tid < rows_cap) {
        int g = order ? order[first + tid] : first + tid;
        sup[tid] = g;
        wg_store(&g2l[g], tid);
    }
    if (tid == 0) { s_size[0] = Bt; s_flag[0] = 0; }
    __syncthreads();
    if (Bt > rows_cap) {
        for (int t = tid; t < rows_cap; t += WGT) wg_store(&g2l[sup[t]], UNSEEN);
        __syncthreads();
        return -1;
    }
    tile_positions(rad, sup, Bt, s_tp);
    __syncthreads();
    for (int k = 1; k <= K; ++k) {
        const int begin = (k >= 2) ? s_size[k - 2] : 0, end = s_size[k - 1];
        const long nent = (long)(end - begin) * deg_max;
        for (long e = tid; e < nent; e += WGT) {
            int t = begin + (int)(e / deg_max), s = (int)(e % deg_max);
            int g = sup[t];
            int p0 = row_ptr[g], deg = row_ptr[g + 1] - p0;
            if (s < deg) {
                const int j = nbr_j[p0 + s];
                if (inside_any(rad, j, s_tp, Bt)) wg_min(&g2l[j], CLAIM + (int)e);
            }
        }
        __syncthreads();
        int base = end;
        for (long c0 = 0; c0 < nent; c0 += WGT) {
            long e = c0 + tid;
            int own = 0, j = -1;
            if (e < nent) {
                int t = begin + (int)(e / deg_max), s = (int)(e % deg_max);
                int g = sup[t];
                int p0 = row_ptr[g], deg = row_ptr[g + 1] - p0;
                if (s < deg) {
                    j = nbr_j[p0 + s];
                    own = wg_load(&g2l[j]) == CLAIM + (int)e;
                }
            }
            int tot;
            int pos = wg_scan01<WGT>(own, s_wave, tot);
            if (own) {
                int idx = base + pos;
                if (idx < rows_cap) { sup[idx] = j; wg_store(&g2l[j], idx); }
                else s_flag[0] = 1;
            }
            base += tot;
        }
        __syncthreads();
        if (s_flag[0]) {
            // restore the map: every claimed atom neighbours this frontier
            for (int t = tid; t < min(base, rows_cap); t += WGT) wg_store(&g2l[sup[t]], UNSEEN);
            for (long e = tid; e < nent; e += WGT) {
                int t = begin + (int)(e / deg_max), s = (int)(e % deg_max);
                int g = sup[t];
                int p0 = row_ptr[g], deg = row_ptr[g + 1] - p0;
                if (s < deg) wg_store(&g2l[nbr_j[p0 + s]], UNSEEN);
            }
            __syncthreads();
            return -1;
        }
        if (tid == 0) s_size[k] = base;
        __syncthreads();
    }
    return s_size[K];
}

// the plan's largest support per step (the moment launches are sized by it)
struct RowsK {
    int r[MAXK + 1];
};

// rows with at most this many neighbours classify their slots in one sweep
constexpr int PREP_REG = 24;

// exclusive prefix of v over the workgroup (thread order); writes the total
constexpr int FRONT = 1024;      // frontier rows per chunk of the bitmap search

template <int WGT>
__device__ inline int wg_scan_excl(int v, int *s_wave, int &total)
{
    constexpr int NW = WGT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(inc, o);
        if (lane >= o) inc += u;
    }
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        const int c = s_wave[q];
        off += (q < w) ? c : 0;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

// The same search with two bitmaps in LDS (one bit per atom): visited atoms,
// and the atoms found for the current layer.  Each frontier (row, slot) sets
// its neighbour's bit in the layer bitmap unless visited; the layer is then
// listed in ascending atom index by a scan of that bitmap, so the row order
// does not depend on scheduling.  g2l gets the local rows as in bfs_tile.
// Both bitmaps are all zero on entry and on return.
template <int WGT>
__device__ int bfs_tile_bits(int tile, int B, int n_atoms, int K, const int *__restrict__ order,
                             const int *__restrict__ row_ptr, const int *__restrict__ nbr_j, int deg_max,
                             int *g2l, int *sup, int rows_cap, int *s_size, int *s_wave, unsigned *s_vis,
                             unsigned *s_new, int nw, int *s_p0, int *s_deg, const Radius &rad, double *s_tp)
{
    const int tid = threadIdx.x;
    const int first = tile * B;
    const int Bt = min(B, n_atoms - first);
    if (tid < Bt && tid < rows_cap) {
        const int g = order ? order[first + tid] : first + tid;
        sup[tid] = g;
        if (Bt <= rows_cap) {
            wg_store(&g2l[g], tid);
            atomicOr(&s_vis[g >> 5], 1u << (g & 31));
        }
    }
    if (tid == 0) s_size[0] = Bt;
    __syncthreads();
    if (Bt > rows_cap) return -1;
    tile_positions(rad, sup, Bt, s_tp);
    __syncthreads();
    const int per = (nw + WGT - 1) / WGT;
    const int w0 = min(tid * per, nw), w1 = min(w0 + per, nw);
    for (int k = 1; k <= K; ++k) {
        const int begin = (k >= 2) ? s_size[k - 2] : 0, end = s_size[k - 1];
        // frontier rows in chunks of FRONT: each row's pair range is looked up
        // once into LDS, then every (row, slot) entry needs one load
        for (int c0 = begin; c0 < end; c0 += FRONT) {
            const int c1 = min(end, c0 + FRONT);
            for (int t = c0 + tid; t < c1; t += WGT) {
                const int g = sup[t];
                const int p0 = row_ptr[g];
                s_p0[t - c0] = p0;
                s_deg[t - c0] = row_ptr[g + 1] - p0;
            }
            __syncthreads();
            const long nent = (long)(c1 - c0) * deg_max;
            for (long e = tid; e < nent; e += WGT) {
                const int tl = (int)(e / deg_max), sl = (int)(e % deg_max);
                if (sl < s_deg[tl]) {
                    const int j = nbr_j[s_p0[tl] + sl];
                    const unsigned bit = 1u << (j & 31);
                    if (!(s_vis[j >> 5] & bit) && inside_any(rad, j, s_tp, Bt)) atomicOr(&s_new[j >> 5], bit);
                }
            }
            __syncthreads();
        }
        int cnt = 0;
        for (int w = w0; w < w1; ++w) cnt += __popc(s_new[w]);
        int tot;
        int idx = end + wg_scan_excl<WGT>(cnt, s_wave, tot);
        const bool over = end + tot > rows_cap;
        for (int w = w0; w < w1; ++w) {
            unsigned m = s_new[w];
            if (!m) continue;
            s_new[w] = 0u;
            s_vis[w] |= m;
            if (over) continue;
            while (m) {
                const int j = w * 32 + (__ffs(m) - 1);
                m &= m - 1u;
                sup[idx] = j;
                wg_store(&g2l[j], idx);
                ++idx;
            }
        }
        __syncthreads();
        if (over) {
            for (int w = tid; w < nw; w += WGT) s_vis[w] = 0u;
            for (int t = tid; t < end; t += WGT) wg_store(&g2l[sup[t]], UNSEEN);
            __syncthreads();
            return -1;
        }
        if (tid == 0) s_size[k] = end + tot;
        __syncthreads();
    }
    const int rows = s_size[K];
    for (int t = tid; t < rows; t += WGT) s_vis[sup[t] >> 5] = 0u;
    __syncthreads();
    return rows;
}

template <int WGT>
__device__ inline void reset_map(int *g2l, const int *sup, int rows)
{
    for (int t = threadIdx.x; t < rows; t += WGT) wg_store(&g2l[sup[t]], UNSEEN);
    __syncthreads();
}

__device__ inline int next_tile(int *queue, int *s_tile)
{
    if (threadIdx.x == 0) s_tile[0] = atomicAdd(queue, 1);
    __syncthreads();
    int t = s_tile[0];
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------------
// plan pass: support sizes only
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(PLAN_T)
k_plan(int n_atoms, int B, int n_tiles, int K, const int *__restrict__ order,
       const int *__restrict__ row_ptr, const int *__restrict__ nbr_j, int deg_max,
       int *hdr, char *scratch, size_t per_wg, Radius rad)
{
    __shared__ int s_size[MAXK + 2], s_wave[PLAN_T / 64], s_flag[1], s_tile[1];
    __shared__ double s_tp[3 * 64];
    char *mine = scratch + per_wg * blockIdx.x;
    int *g2l = (int *)mine;
    int *sup = (int *)(mine + align_up(4ull * n_atoms, 256));
    for (;;) {
        int tile = next_tile(&hdr[0], s_tile);
        if (tile >= n_tiles) break;
        int rows = bfs_tile<PLAN_T>(tile, B, n_atoms, K, order, row_ptr, nbr_j, deg_max, g2l, sup,
                                    n_atoms, s_size, s_wave, s_flag, rad, s_tp);
        if (threadIdx.x <= K) atomicMax(&hdr[8 + threadIdx.x], s_size[threadIdx.x]);
        if (threadIdx.x == 0) atomicMax(&hdr[2], rows);
        reset_map<PLAN_T>(g2l, sup, rows);
    }
}

// Plan pass with a visited bitmap in LDS (systems small enough for one bit
// per atom in a workgroup's LDS).  The layer sizes do not depend on the order
// in which a layer's atoms are found, so each frontier entry claims its
// neighbour with one LDS atomic OR and the new atoms are appended in any order
// (a wave-level ballot and one LDS counter), instead of the ordered claim and
// compaction the prepare pass needs.
__global__ void __launch_bounds__(PLAN_T)
k_plan_bits(int n_atoms, int B, int n_tiles, int K, const int *__restrict__ order,
            const int *__restrict__ row_ptr, const int *__restrict__ nbr_j, int deg_max,
            int *hdr, char *scratch, size_t per_wg, Radius rad)
{
    extern __shared__ unsigned s_bits[];
    __shared__ int s_size[MAXK + 2], s_tile[1], s_cnt[1], s_p0[FRONT], s_deg[FRONT];
    __shared__ double s_tp[3 * 64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int nw = (n_atoms + 31) / 32;
    for (int i = tid; i < nw; i += PLAN_T) s_bits[i] = 0u;
    __syncthreads();
    int *sup = (int *)(scratch + per_wg * blockIdx.x);
    for (;;) {
        const int tile = next_tile(&hdr[0], s_tile);
        if (tile >= n_tiles) break;
        const int first = tile * B, Bt = min(B, n_atoms - first);
        if (tid < Bt) {
            const int g = order ? order[first + tid] : first + tid;
            sup[tid] = g;
            atomicOr(&s_bits[g >> 5], 1u << (g & 31));
        }
        if (tid == 0) { s_size[0] = Bt; s_cnt[0] = Bt; }
        __syncthreads();
        tile_positions(rad, sup, Bt, s_tp);
        __syncthreads();
        for (int k = 1; k <= K; ++k) {
            const int begin = (k >= 2) ? s_size[k - 2] : 0, end = s_size[k - 1];
            // frontier rows in chunks of FRONT, their pair ranges looked up once
            for (int f0 = begin; f0 < end; f0 += FRONT) {
                const int f1 = min(end, f0 + FRONT);
                for (int t = f0 + tid; t < f1; t += PLAN_T) {
                    const int g = sup[t];
                    const int p0 = row_ptr[g];
                    s_p0[t - f0] = p0;
                    s_deg[t - f0] = row_ptr[g + 1] - p0;
                }
                __syncthreads();
                const long nent = (long)(f1 - f0) * deg_max;
                for (long c0 = 0; c0 < nent; c0 += PLAN_T) {
                    const long e = c0 + tid;
                    int j = -1;
                    bool fresh = false;
                    if (e < nent) {
                        const int tl = (int)(e / deg_max), sl = (int)(e % deg_max);
                        if (sl < s_deg[tl]) {
                            j = nbr_j[s_p0[tl] + sl];
                            const unsigned bit = 1u << (j & 31);
                            if (!(s_bits[j >> 5] & bit) && inside_any(rad, j, s_tp, Bt))
                                fresh = !(atomicOr(&s_bits[j >> 5], bit) & bit);
                        }
                    }
                    const unsigned long long m = __ballot(fresh);
                    int at = 0;
                    if (lane == 0 && m) at = atomicAdd(&s_cnt[0], (int)__popcll(m));
                    at = __shfl(at, 0);
                    if (fresh) sup[at + __popcll(m & ((1ull << lane) - 1ull))] = j;
                }
                __syncthreads();
            }
            if (tid == 0) s_size[k] = s_cnt[0];
            __syncthreads();
        }
        const int rows = s_size[K];
        if (tid <= K) atomicMax(&hdr[8 + tid], s_size[tid]);
        if (tid == 0) atomicMax(&hdr[2], rows);
        for (int t = tid; t < rows; t += PLAN_T) s_bits[sup[t] >> 5] = 0u;
        __syncthreads();
    }
}

__global__ void k_max_degree(int n, const int *__restrict__ row_ptr, int *hdr)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int d = (i < n) ? row_ptr[i + 1] - row_ptr[i] : 0;
    for (int o = 32; o > 0; o >>= 1) d = max(d, __shfl_xor(d, o));
    if ((threadIdx.x & 63) == 0) atomicMax(&hdr[3], d);
}

__global__ void k_init(int *hdr, int n_hdr, int *maps, long n_map)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_hdr) hdr[i] = 0;
    if (i < n_map) maps[i] = UNSEEN;
}

// ---------------------------------------------------------------------------
// prepare pass: supports, layers and layer-sorted neighbour slots of every tile
// ---------------------------------------------------------------------------
template <bool BITS>
__global__ void __launch_bounds__(PLAN_T)
k_prepare(int n_atoms, int B, int n_tiles, int K, const int *__restrict__ order,
          const int *__restrict__ row_ptr, const int *__restrict__ nbr_j, int deg_max, int rows_cap,
          RowsK rows_k, int *hdr, char *ws, Layout lay, size_t map_stride, Radius rad)
{
    __shared__ int s_size[MAXK + 2], s_wave[PLAN_T / 64], s_flag[1], s_tile[1];
    __shared__ double s_tp[3 * 64];
    __shared__ int s_p0[BITS ? FRONT : 1], s_deg[BITS ? FRONT : 1];
    extern __shared__ unsigned s_bits2[];        // BITS: visited and layer bitmaps
    const int nw = (n_atoms + 31) / 32;
    if constexpr (BITS) {
        for (int i = threadIdx.x; i < 2 * nw; i += PLAN_T) s_bits2[i] = 0u;
        __syncthreads();
    }
    int *g2l = (int *)(ws + lay.x + map_stride * blockIdx.x);
    int *sizes = (int *)(ws + lay.sizes);
    for (;;) {
        const int tile = next_tile(&hdr[0], s_tile);
        if (tile >= n_tiles) break;
        char *tb = ws + lay.tiles + lay.tile_stride * tile;
        int *sup = (int *)tb;
        int *rinfo = sup + rows_cap;
        int *lnb = rinfo + rows_cap;
        const int rows = BITS ? bfs_tile_bits<PLAN_T>(tile, B, n_atoms, K, order, row_ptr, nbr_j, deg_max, g2l,
                                                      sup, rows_cap, s_size, s_wave, s_bits2, s_bits2 + nw, nw,
                                                      s_p0, s_deg, rad, s_tp)
                              : bfs_tile<PLAN_T>(tile, B, n_atoms, K, order, row_ptr, nbr_j, deg_max, g2l, sup,
                                                 rows_cap, s_size, s_wave, s_flag, rad, s_tp);
        if (rows < 0) {
            // support larger than planned: keep the seeds so that their moments
            // can be marked NaN, and raise the error flag
            if (threadIdx.x == 0) {
                sizes[tile * (MAXK + 2)] = -1;
                sizes[tile * (MAXK + 2) + 1] = min(min(B, n_atoms - tile * B), rows_cap);
                atomicOr(&hdr[1], 1);
            }
            __syncthreads();
            continue;
        }
        if (threadIdx.x <= K) sizes[tile * (MAXK + 2) + threadIdx.x] = s_size[threadIdx.x];
        // a support larger at some step than the plan's largest (the launches
        // are sized by those) also fails the tile
        if (threadIdx.x == 0) {
            int over = 0;
            for (int k = 0; k <= K; ++k) over |= s_size[k] > rows_k.r[k];
            s_flag[0] = over;
        }
        __syncthreads();
        // per row: neighbour slots by class (0: layer < L, 1: layer L, 2: layer
        // L + 1, 3: outside the support), stable in slot order within a class;
        // one sweep counts, a second places, slot loads issued eight at a time
        for (int l = threadIdx.x; l < rows; l += PLAN_T) {
            const int g = sup[l];
            int L = 0;
            while (l >= s_size[L]) ++L;
            const int lo = (L >= 1) ? s_size[L - 1] : 0;   // rows of layers < L
            const int endL = s_size[L];
            const int endL1 = (L + 1 <= K) ? s_size[L + 1] : s_size[K];
            const int p0 = row_ptr[g], deg = row_ptr[g + 1] - p0;
            if (deg > deg_max) {        // more neighbours than planned: the tile fails
                s_flag[0] = 1;
                continue;
            }
            int *dst = lnb + (long)l * deg_max;
            int cnt[3] = {0, 0, 0};
            if (deg <= PREP_REG) {
                // one sweep: all slots' local rows in registers, then count and place
                int lj[PREP_REG];
#pragma unroll
                for (int u = 0; u < PREP_REG; ++u) lj[u] = (u < deg) ? nbr_j[p0 + u] : -1;
#pragma unroll
                for (int u = 0; u < PREP_REG; ++u) lj[u] = lj[u] >= 0 ? wg_load(&g2l[lj[u]]) : UNSEEN;
                int cls[PREP_REG];
#pragma unroll
                for (int u = 0; u < PREP_REG; ++u) {
                    cls[u] = (lj[u] < lo) ? 0 : (lj[u] < endL ? 1 : (lj[u] < endL1 ? 2 : 3));
                    cnt[0] += cls[u] == 0;
                    cnt[1] += cls[u] == 1;
                    cnt[2] += cls[u] == 2;
                }
                int o[3] = {0, cnt[0], cnt[0] + cnt[1]};
#pragma unroll
                for (int u = 0; u < PREP_REG; ++u) {
                    if (cls[u] == 0) dst[o[0]++] = (lj[u] << 8) | u;
                    else if (cls[u] == 1) dst[o[1]++] = (lj[u] << 8) | u;
                    else if (cls[u] == 2) dst[o[2]++] = (lj[u] << 8) | u;
                }
            } else
            for (int pass = 0; pass < 2; ++pass) {
                int o[3] = {0, cnt[0], cnt[0] + cnt[1]};
                for (int s0 = 0; s0 < deg; s0 += 8) {
                    int lj[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) lj[u] = (s0 + u < deg) ? nbr_j[p0 + s0 + u] : -1;
#pragma unroll
                    for (int u = 0; u < 8; ++u) lj[u] = lj[u] >= 0 ? wg_load(&g2l[lj[u]]) : UNSEEN;
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int cls = (lj[u] < lo) ? 0 : (lj[u] < endL ? 1 : (lj[u] < endL1 ? 2 : 3));
                        if (cls < 3) {
                            if (pass == 0) ++cnt[cls];
                            else dst[o[cls]++] = (lj[u] << 8) | (s0 + u);
                        }
                    }
                }
            }
            const int n1 = cnt[0], n2 = cnt[0] + cnt[1], c = n2 + cnt[2];
            rinfo[l] = L | (n1 << 8) | (n2 << 16) | (c << 24);
            if (rad.on) {
                // the columns of tile atom t keep this row if it lies within r_max of t
                int *rmask = lnb + (long)rows_cap * deg_max;
                const int Bt = s_size[0];
                const double pj[3] = {rad.pos[3 * (long)g], rad.pos[3 * (long)g + 1], rad.pos[3 * (long)g + 2]};
                int bits = 0;
                for (int t = 0; t < Bt; ++t)
                    if (within(rad, pj, s_tp + 3 * t)) bits |= 1 << t;
                rmask[l] = bits;
            }
        }
        __syncthreads();
        if (s_flag[0] && threadIdx.x == 0) {
            sizes[tile * (MAXK + 2)] = -1;
            sizes[tile * (MAXK + 2) + 1] = min(min(B, n_atoms - tile * B), rows_cap);
            atomicOr(&hdr[1], 1);
        }
        reset_map<PLAN_T>(g2l, sup, rows);
    }
}

// ---------------------------------------------------------------------------
// moments: X^0, steps, reductions
// ---------------------------------------------------------------------------
template <typename T> __device__ inline T from_f64(double v) { return (T)v; }

struct Batch {
    int first, count;          // tiles [first, first + count)
};

// X^0 = unit columns on the seed rows; mu_0 = 1 (NaN moments for failed tiles)
template <typename T, int NO>
__global__ void k_x0(Batch bt, int n_max, int B, const int *__restrict__ sizes_, const char *tiles_base,
                     size_t tile_stride, char *xbase, size_t x_stride, double *__restrict__ mu)
{
    const int t = blockIdx.x;
    if (t >= bt.count) return;
    const int tile = bt.first + t;
    const int *sizes = sizes_ + tile * (MAXK + 2);
    const int *sup = (const int *)(tiles_base + tile_stride * tile);
    const int n1m = n_max + 1;
    if (sizes[0] < 0) {          // failed tile: NaN moments for its seeds
        for (int e = threadIdx.x; e < sizes[1] * NO * n1m; e += blockDim.x) {
            int b = e / (NO * n1m), rest = e % (NO * n1m);
            mu[(long)sup[b] * NO * n1m + rest] = __builtin_nan("");
        }
        return;
    }
    const int Bt = sizes[0];
    T *X0 = (T *)(xbase + x_stride * (2 * (size_t)t));
    for (int e = threadIdx.x; e < Bt * NO * 64; e += blockDim.x) {
        int l = e / (NO * 64), rest = e % (NO * 64), a = rest / 64, c = rest % 64;
        X0[(long)l * NO * 64 + a * 64 + c] = (c == l * NO + a) ? T(1) : T(0);
    }
    for (int e = threadIdx.x; e < Bt * NO; e += blockDim.x) {
        int b = e / NO, a = e % NO;
        mu[((long)sup[b] * NO + a) * n1m] = 1.0;
    }
}

// Asynchronous copy of n floats from global memory into an LDS slice
// (global_load_lds: lane i's dword lands at the slice base + 4 i for every
// 64-float chunk); completion is counted by vmcnt like any vector load.
__device__ inline void h_to_lds(const float *src, float *dst, int n, int lane)
{
    for (int e = 0; e < n; e += 64)
        if (e + lane < n)
            __builtin_amdgcn_global_load_lds((const void *)(src + e + lane),
                                             (__attribute__((address_space(3))) void *)(dst + e), 4, 0, 0);
}

// The same copy 16 bytes per lane (global_load_lds_dwordx4: lane i's 16 bytes
// land at the slice base + 16 i for every 256-float chunk); n a multiple of 4,
// src and dst 16-byte aligned.  One instruction moves 1 KB.
__device__ inline void h_to_lds16(const float *src, float *dst, int n, int lane)
{
    for (int e = 0; e < n; e += 256)
        if (e + 4 * lane < n)
            __builtin_amdgcn_global_load_lds((const void *)(src + e + 4 * lane),
                                             (__attribute__((address_space(3))) void *)(dst + e), 16, 0, 0);
}

// read-only arrays seen through the constant address space, so that loads at
// wave-uniform addresses (a row's atom, layer word, pair range, onsite levels)
// become scalar loads instead of vector loads that every lane repeats
template <typename T> __device__ inline const __attribute__((address_space(4))) T *cst(const T *p)
{
    return (const __attribute__((address_space(4))) T *)p;
}

// Floats of one wave's LDS slice of H blocks (deg_max blocks, whole 64-float
// chunks so that the copy never writes past it).
__host__ __device__ inline int h_slice(int deg_max, int nb) { return (deg_max * nb + 63) / 64 * 64; }

// One step (or the final odd H X^K pass) for a batch of tiles.
// Latency structure: the H blocks of a wave's next row (one contiguous range
// of pairs) are copied into its LDS slice asynchronously as soon as the
// current row's products are done, so they arrive with the next row's first
// gathers; the X gathers of G neighbour slots are issued before any of them is
// used, so a row costs a few memory round trips instead of one per slot.  X^k
// is written with non-temporal stores: it is read only by the next launch,
// long after it would have left L2, where it would evict the rows being
// gathered.
//
// LANCZOS = 1: one whole Lanczos level j = k - 1 per pass (the support of
// H u_j is that of X^k).  A tile then has four vectors: Y (two, ping-pong) and
// R (two).  Entering the pass, Y holds y'_j = H u_(j-1) - b_(j-1) u_(j-2) (not
// yet orthogonalised against u_(j-1)) and R holds r_(j-1), r_(j-2), with
// u = s r.  The gathers read Y only: H r_j = H y'_j - c_j H r_(j-1), c_j =
// a_(j-1) s_(j-1), and H r_(j-1) = (y'_j + beta_(j-1) r_(j-2)) / s_(j-1) is a
// combination of the row's own entries, so no second vector is gathered and
// no separate update pass is needed.  Per row the pass forms
//   r_j = y'_j - c_j r_(j-1)            (stored in place of r_(j-2)),
//   y'_(j+1) = s_j H r_j - beta_j r_(j-1)  (stored in the other Y buffer),
// and partial sums of <r_j, y'_(j+1)>, |y'_(j+1)|^2 and |r_j|^2, from which
// k_lreduce_fused takes a_j = s_j <r_j, y'_(j+1)> and b_(j+1)^2 = |y'_(j+1) -
// a_j u_j|^2 = |y'|^2 - 2 a_j^2 + a_j^2 s_j^2 |r_j|^2.  Per column (lane) lc
// gives s_j, beta_j = b_j s_(j-1), c_j, beta_(j-1) and 1/s_(j-1).
template <typename T, int NO, int WGT, int LANCZOS, typename S = T, bool HS = false, bool TR = false>
__global__ void __launch_bounds__(WGT)
k_step(Batch bt, int k, int K, int last, int keep, int fin, int nch, int chunk_rows, int deg_max, int rows_cap,
       const int *__restrict__ row_ptr, const double *__restrict__ H_on, const T *__restrict__ H,
       const int *__restrict__ sizes_, const char *tiles_base, size_t tile_stride, char *xbase,
       size_t x_stride, double *__restrict__ part, const double *__restrict__ lc)
{
    constexpr int NW = WGT / 64;
    // values per H block: d-d blocks are stored packed (symmetric, upper
    // triangle), s,p,d blocks in full
    constexpr int NB = NO == 5 ? BOP_D_PACKED : NO * NO;
    // Slots whose gathers are in flight together.  Occupancy decides the step:
    // FP32 takes groups of 2 slots, double-buffered (the next group's gathers
    // are issued before the current one is multiplied), which keeps the d
    // kernel at 59 VGPRs (8 waves per SIMD) and measured 3% faster than single
    // groups of 4 and 8% faster than double-buffered groups of 4 (6 waves);
    // FP64 rows are two or four times wider, and single groups of 2 (d) or
    // 1 (s,p,d) slots measured fastest there.
    constexpr bool PIPE = sizeof(T) == 4;
    constexpr int G = sizeof(T) == 8 ? (NO <= 5 ? 2 : 1) : 2;
    __shared__ double s_red[LANCZOS ? 3 : 2][NW][64];
    extern __shared__ char s_dyn[];
    // XCD-aware numbering: block b runs on XCD b % 8; the other factor walks
    // tile-major through (tile, chunk)
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int t = (q / nch) * 8 + xcd, chunk = q % nch;
    if (t >= bt.count) return;
    const int tile = bt.first + t;
    const int *sizes = sizes_ + tile * (MAXK + 2);
    if (sizes[0] < 0) return;
    const int nrow = last ? sizes[K] : sizes[k];
    const int nct = tile_chunks(nrow, chunk_rows, NW);
    if (chunk >= nct) return;
    const int RS = nct * NW;                                 // row stride of this chunk
    const int *sup = (const int *)(tiles_base + tile_stride * tile);
    const int *rinfo = sup + rows_cap;
    const int *lnb = rinfo + rows_cap;
    const int *rmask = lnb + (long)rows_cap * deg_max;   // path radius: tile atoms that keep the row
    const int src = last ? (K & 1) : ((k - 1) & 1);
    constexpr size_t NBUF = LANCZOS ? 4 : 2;      // X buffers per tile
    const S *Xp = (const S *)(xbase + x_stride * (NBUF * t + src));
    S *Xc = (S *)(xbase + x_stride * (NBUF * t + (k & 1)));
    // Lanczos: r_(j-2) read and r_j written (same buffer), r_(j-1) read
    S *Ra = (S *)(xbase + x_stride * (NBUF * t + 2 + ((k - 1) & 1)));
    const S *Rb = (const S *)(xbase + x_stride * (NBUF * t + 2 + (k & 1)));
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    T *sH = (T *)s_dyn + (size_t)w * h_slice(deg_max, NB);  // this wave's H blocks
    constexpr int stride_row = NO * 64;
    double so = 0.0, se = 0.0, sx = 0.0;
    T ls = T(1), lbeta = T(0), lcj = T(0), lbp = T(0), linv = T(0);
    if (LANCZOS) {
        const double *l = lc + (size_t)t * LC_N * 64 + lane;
        ls = (T)l[0];
        lbeta = (T)l[64];
        lcj = (T)l[128];
        lbp = (T)l[192];
        linv = (T)l[256];
    }
    // a row's H blocks into the LDS slice: 16 bytes per lane where every block
    // is a whole number of 16-byte units (packed FP32 d-d blocks, 64 bytes)
    auto h_copy = [&](const float *src, float *dst, int n) {
        if constexpr (sizeof(T) == 4 && (NB * sizeof(T)) % 16 == 0) h_to_lds16(src, dst, n, lane);
        else h_to_lds(src, dst, n, lane);
    };
    // the next row's atom, layer word, slot list and pair range are fetched while
    // the current row computes, which takes their dependent loads off the
    // critical path
    int l = chunk * NW + w;
    int g_n = 0, info_n = 0, slots_n = 0, p0_n = 0, p1_n = 0, tm_n = -1;
    if (l < nrow) {
        g_n = cst(sup)[l];
        info_n = cst(rinfo)[l];
        if constexpr (TR) tm_n = cst(rmask)[l];
        slots_n = lane < deg_max ? lnb[(long)l * deg_max + lane] : 0;
        p0_n = cst(row_ptr)[g_n];
        p1_n = cst(row_ptr)[g_n + 1];
        if constexpr (!HS) h_copy((const float *)(H + (long)p0_n * NB), (float *)sH, (p1_n - p0_n) * NB);
    }
    for (; l < nrow; l += RS) {
        const int g = g_n, info = info_n, slots_all = slots_n, p0 = p0_n, deg = p1_n - p0_n, tm = tm_n;
        if (l + RS < nrow) {
            g_n = cst(sup)[l + RS];
            info_n = cst(rinfo)[l + RS];
            if constexpr (TR) tm_n = cst(rmask)[l + RS];
            slots_n = lane < deg_max ? lnb[(long)(l + RS) * deg_max + lane] : 0;
            p0_n = cst(row_ptr)[g_n];
            p1_n = cst(row_ptr)[g_n + 1];
        }
        const int L = info & 255, n1 = (info >> 8) & 255, n2 = (info >> 16) & 255, n3 = (info >> 24) & 255;
        const bool has_prev = last || L <= k - 1;
        const int nval = last ? n3 : (k - 1 >= L + 1 ? n3 : (k - 1 == L ? n2 : n1));
        const int slots = (lane < nval) ? slots_all : 0;
        // the row's H blocks (contiguous pairs p0 .. p0 + deg): in the LDS slice
        // (copied there after the previous row), or (HS) read with scalar loads
        // straight into SGPR operands from their wave-uniform addresses.  HS
        // measured 11-34% faster for FP64 and slower for FP32; FP32 uses it only
        // where the LDS slice would not fit a workgroup.
        constexpr bool H_SCALAR = HS;
        const T *hsrc = H + (long)p0 * NB;
        (void)deg;
        const S *xrow = Xp + (long)l * stride_row + lane;
        T acc[NO], xs[NO], r1[LANCZOS ? NO : 1], r2[LANCZOS ? NO : 1];
#pragma unroll
        for (int a = 0; a < NO; ++a) {
            xs[a] = has_prev ? (T)xrow[a * 64] : T(0);
            acc[a] = from_f64<T>(cst(H_on)[(long)g * NO + a]) * xs[a];
        }
        // gather a group of G slots (slots past nval re-read this row, harmless,
        // and are masked in the product)
        auto gather = [&](int s0, T (&x)[G][NO], int (&hoff)[G]) {
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int su = s0 + u < nval ? s0 + u : 0;
                const int pk = __builtin_amdgcn_readlane(slots, su);
                const S *xn = (s0 + u < nval) ? Xp + (long)(pk >> 8) * stride_row + lane : xrow;
                hoff[u] = (pk & 255) * NB;
#pragma unroll
                for (int b = 0; b < NO; ++b) x[u][b] = (T)xn[b * 64];
            }
        };
        auto product = [&](int s0, const T (&x)[G][NO], const int (&hoff)[G]) {
#pragma unroll
            for (int u = 0; u < G; ++u) {
                if (s0 + u < nval) {
                    const T *h = H_SCALAR ? hsrc + hoff[u] : sH + hoff[u];
#pragma unroll
                    for (int a = 0; a < NO; ++a)
#pragma unroll
                        for (int b = 0; b < NO; ++b)
                            acc[a] = fma(h[NO == 5 ? d_packed_index(a, b) : a * NO + b], x[u][b], acc[a]);
                }
            }
        };
        auto h_ready = [&]() {
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_s_waitcnt(0);      // the row's H blocks have reached LDS
            __builtin_amdgcn_wave_barrier();
        };
        if constexpr (PIPE) {
            T xa[G][NO], xb[G][NO];
            int ha[G], hb[G];
            if (nval > 0) {
                gather(0, xa, ha);
                h_ready();
            }
            for (int s0 = 0; s0 < nval; s0 += 2 * G) {
                if (s0 + G < nval) gather(s0 + G, xb, hb);
                product(s0, xa, ha);
                if (s0 + G < nval) {
                    if (s0 + 2 * G < nval) gather(s0 + 2 * G, xa, ha);
                    product(s0 + G, xb, hb);
                }
            }
        } else {
            for (int s0 = 0; s0 < nval; s0 += G) {
                T x[G][NO];
                int hoff[G];
                gather(s0, x, hoff);
                if (s0 == 0) h_ready();
                product(s0, x, hoff);
            }
        }
        // path radius: a column keeps the row only within r_max of its atom
        if constexpr (TR) {
            if (!((tm >> (lane / NO)) & 1)) {
#pragma unroll
                for (int a = 0; a < NO; ++a) acc[a] = T(0);
            }
        }
        (void)tm;
        __builtin_amdgcn_wave_barrier();   // all lanes done with sH before the next row's copy
        if constexpr (!HS) {
            if (nval == 0) __builtin_amdgcn_s_waitcnt(0);   // this row's copy (unused) has landed
            if (l + RS < nrow) h_copy((const float *)(H + (long)p0_n * NB), (float *)sH, (p1_n - p0_n) * NB);
        }
        S *xo = Xc + (long)l * stride_row + lane;
        if constexpr (LANCZOS) {
            // the row's own r_(j-1) and r_(j-2) (zero outside their supports),
            // loaded after the products so that they hold no registers there;
            // read once, so non-temporal loads keep them from displacing the
            // gathered rows in L2 (1% on the FP32 pass)
            const bool h1 = L <= k - 2, h2 = L <= k - 3;
            const long off = (long)l * stride_row + lane;
#pragma unroll
            for (int a = 0; a < NO; ++a) {
                r1[a] = h1 ? (T)__builtin_nontemporal_load(&Rb[off + a * 64]) : T(0);
                r2[a] = h2 ? (T)__builtin_nontemporal_load(&Ra[off + a * 64]) : T(0);
            }
            S *ro = Ra + (long)l * stride_row + lane;
#pragma unroll
            for (int a = 0; a < NO; ++a) {
                const T hrp = (xs[a] + lbp * r2[a]) * linv;      // H r_(j-1) at this row
                const T hr = acc[a] - lcj * hrp;                 // H r_j
                const S rj = (S)(xs[a] - lcj * r1[a]);           // r_j
                const S y = (S)(ls * hr - lbeta * r1[a]);        // y'_(j+1)
                // r_j is zero on the newest layer (L = k, where y'_j and r_(j-1)
                // are) and no later pass reads it there: stored on the older
                // layers only
                if (keep) {
                    if (has_prev) __builtin_nontemporal_store(rj, &ro[a * 64]);
                    __builtin_nontemporal_store(y, &xo[a * 64]);
                }
                // sums of the vectors as stored
                const double rd = (double)(T)rj, yd = (double)(T)y;
                so = fma(rd, yd, so);
                se = fma(yd, yd, se);
                sx = fma(rd, rd, sx);
            }
        } else {
            if (keep) {
#pragma unroll
                for (int a = 0; a < NO; ++a) __builtin_nontemporal_store((S)acc[a], &xo[a * 64]);
            }
#pragma unroll
            for (int a = 0; a < NO; ++a) {
                so = fma((double)xs[a], (double)acc[a], so);
                se = fma((double)acc[a], (double)acc[a], se);
            }
        }
    }
    s_red[0][w][lane] = so;
    s_red[1][w][lane] = se;
    if constexpr (LANCZOS) s_red[2][w][lane] = sx;
    __syncthreads();
    if (threadIdx.x < 64) {
        double to = 0.0, te = 0.0, tx = 0.0;
#pragma unroll
        for (int q2 = 0; q2 < NW; ++q2) {
            to += s_red[0][q2][threadIdx.x];
            te += s_red[1][q2][threadIdx.x];
            if constexpr (LANCZOS) tx += s_red[2][q2][threadIdx.x];
        }
        constexpr int ns = LANCZOS ? 3 : 2;
        double *pp = part + (((size_t)t * nch + chunk) * ns) * 64;
        pp[threadIdx.x] = to;
        pp[64 + threadIdx.x] = te;
        if constexpr (LANCZOS) pp[128 + threadIdx.x] = tx;
    }
}

// mu[.][2k-1], mu[.][2k] (or mu[.][2K+1]) from the chunk partials, in chunk
// order; one launch after a batch's last step, block (tile, step k - 1)
template <int NO>
__global__ void k_reduce(Batch bt, int K, int n_max, StepParts sp, int chunk_rows, int nw,
                         const int *__restrict__ sizes_, const char *tiles_base, size_t tile_stride,
                         const double *__restrict__ part_all, double *__restrict__ mu)
{
    const int t = blockIdx.x;
    const int k = blockIdx.y + 1, last = k > K;
    const int nch = sp.nch[k];
    if (t >= bt.count || nch <= 0) return;
    const double *part = part_all + sp.off[k];
    const int tile = bt.first + t;
    const int *sizes = sizes_ + tile * (MAXK + 2);
    if (sizes[0] < 0) return;
    const int Bt = sizes[0];
    const int c = threadIdx.x;
    if (c >= Bt * NO) return;
    const int nrow = last ? sizes[K] : sizes[k];
    const int used = tile_chunks(nrow, chunk_rows, nw);
    double to = 0.0, te = 0.0;
    // eight chunks' loads in flight, added in chunk order
    for (int q0 = 0; q0 < used; q0 += 8) {
        double vo[8], ve[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double *pp = part + (((size_t)t * nch + min(q0 + u, used - 1)) * 2) * 64;
            vo[u] = pp[c];
            ve[u] = pp[64 + c];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (q0 + u < used) { to += vo[u]; te += ve[u]; }
    }
    const int *sup = (const int *)(tiles_base + tile_stride * tile);
    const int b = c / NO, a = c % NO;
    double *m = mu + ((long)sup[b] * NO + a) * (n_max + 1);
    if (last) m[2 * K + 1] = to;
    else { m[2 * k - 1] = to; m[2 * k] = te; }
}

// ---------------------------------------------------------------------------
// BF16 form: H.X on MFMA (v_mfma_f32_16x16x32_bf16), FP32 accumulation
// ---------------------------------------------------------------------------
// Per row: D[alpha][c] = sum over (slot, beta) of H[slot][alpha][beta] X[ls][beta][c]
// with M = alpha (n_orb of 16 used), N = 16 columns (4 column blocks), K = 32
// (slot, beta) pairs per instruction, beta padded to the slot width SW (8 for
// d, 16 for s,p,d) so that every lane's eight K values come from one slot and
// one 16-byte load.  Layouts (BF16 bits):
//   H  [P][n_orb][SW]          (pad zero; written by bop_build_H)
//   X  [row][64 columns][SW]   (pad zero)
// Lane i holds A[m = i%16][k = 8(i/16)..+7], B[k = 8(i/16)..+7][n = i%16] and
// D[m = 4(i/16)+j][n = i%16], j = 0..3.  The onsite level is applied to the
// FP32 accumulator; moments use the FP32 values of X^k and the stored BF16
// X^(k-1); X^k is rounded to BF16 (nearest even) when stored.
typedef short bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ inline float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ inline unsigned short f32_to_bf16(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);            // round to nearest even
    return (unsigned short)(u >> 16);
}

template <int NO>
__global__ void k_x0_bf16(Batch bt, int n_max, const int *__restrict__ sizes_, const char *tiles_base,
                          size_t tile_stride, char *xbase, size_t x_stride, double *__restrict__ mu)
{
    constexpr int SW = NO <= 8 ? 8 : 16;
    const int t = blockIdx.x;
    if (t >= bt.count) return;
    const int tile = bt.first + t;
    const int *sizes = sizes_ + tile * (MAXK + 2);
    const int *sup = (const int *)(tiles_base + tile_stride * tile);
    const int n1m = n_max + 1;
    if (sizes[0] < 0) {
        for (int e = threadIdx.x; e < sizes[1] * NO * n1m; e += blockDim.x) {
            int b = e / (NO * n1m), rest = e % (NO * n1m);
            mu[(long)sup[b] * NO * n1m + rest] = __builtin_nan("");
        }
        return;
    }
    const int Bt = sizes[0];
    unsigned short *X0 = (unsigned short *)(xbase + x_stride * (2 * (size_t)t));
    for (int e = threadIdx.x; e < Bt * 64 * SW; e += blockDim.x) {
        int l = e / (64 * SW), rest = e % (64 * SW), c = rest / SW, a = rest % SW;
        X0[e] = (a < NO && c == l * NO + a) ? (unsigned short)0x3f80 : (unsigned short)0;
    }
    for (int e = threadIdx.x; e < Bt * NO; e += blockDim.x) {
        int b = e / NO, a = e % NO;
        mu[((long)sup[b] * NO + a) * n1m] = 1.0;
    }
}

// LANCZOS = 1: the Lanczos product of k_step (same column coefficients), with
// r_(k-2) read from the BF16 buffer that y' replaces.
template <int NO, int WGT, int LANCZOS>
__global__ void __launch_bounds__(WGT)
k_step_bf16(Batch bt, int k, int K, int last, int keep, int fin, int nch, int chunk_rows, int deg_max,
            int rows_cap,
            const int *__restrict__ row_ptr, const double *__restrict__ H_on,
            const unsigned short *__restrict__ H, const int *__restrict__ sizes_, const char *tiles_base,
            size_t tile_stride, char *xbase, size_t x_stride, double *__restrict__ part,
            const double *__restrict__ lc)
{
    constexpr int NW = WGT / 64;
    constexpr int SW = NO <= 8 ? 8 : 16;
    constexpr int SPC = 32 / SW;                 // slots per K = 32 chunk
    __shared__ double s_red[LANCZOS ? 3 : 2][NW][64];
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int t = (q / nch) * 8 + xcd, chunk = q % nch;
    if (t >= bt.count) return;
    const int tile = bt.first + t;
    const int *sizes = sizes_ + tile * (MAXK + 2);
    if (sizes[0] < 0) return;
    const int nrow = last ? sizes[K] : sizes[k];
    const int nct = tile_chunks(nrow, chunk_rows, NW);
    if (chunk >= nct) return;
    const int *sup = (const int *)(tiles_base + tile_stride * tile);
    const int *rinfo = sup + rows_cap;
    const int *lnb = rinfo + rows_cap;
    const int src = last ? (K & 1) : ((k - 1) & 1);
    const unsigned short *Xp = (const unsigned short *)(xbase + x_stride * (2 * (size_t)t + src));
    unsigned short *Xc = (unsigned short *)(xbase + x_stride * (2 * (size_t)t + (k & 1)));
    const int lane = threadIdx.x & 63, g = lane >> 4, n = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gslot = (SW == 8) ? g : (g >> 1);  // slot of this lane group within a chunk
    const int boff = (SW == 8) ? 0 : 8 * (g & 1);
    double so[4] = {0, 0, 0, 0}, se[4] = {0, 0, 0, 0}, sx[4] = {0, 0, 0, 0};
    float ls[4] = {1.f, 1.f, 1.f, 1.f}, lbeta[4] = {0.f, 0.f, 0.f, 0.f};
    if (LANCZOS) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            ls[cb] = (float)lc[((size_t)t * LC_N + 0) * 64 + cb * 16 + n];
            lbeta[cb] = (float)lc[((size_t)t * LC_N + 1) * 64 + cb * 16 + n];
        }
    }
    for (int l = chunk * NW + w; l < nrow; l += nct * NW) {
        const int gatom = __builtin_amdgcn_readfirstlane(sup[l]);
        const int info = __builtin_amdgcn_readfirstlane(rinfo[l]);
        const int L = info & 255, n1 = (info >> 8) & 255, n2 = (info >> 16) & 255, n3 = (info >> 24) & 255;
        const bool has_prev = last || L <= k - 1;
        const int nval = last ? n3 : (k - 1 >= L + 1 ? n3 : (k - 1 == L ? n2 : n1));
        const int p0 = row_ptr[gatom];
        const int slots = (lane < nval) ? lnb[(long)l * deg_max + lane] : 0;
        f32x4_t acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        const int nchunk = (nval + SPC - 1) / SPC;
        for (int c0 = 0; c0 < nchunk; c0 += 2) {
            // operands of two K chunks are loaded before either is multiplied
            bf16x8_t a[2], b[2][4];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int sl = (c0 + u) * SPC + gslot;
                const int pk = __shfl(slots, sl < 64 ? sl : 0);
                a[u] = bf16x8_t{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) b[u][cb] = bf16x8_t{0, 0, 0, 0, 0, 0, 0, 0};
                if (sl < nval) {
                    const long ls = pk >> 8, p = p0 + (pk & 255);
                    if (n < NO) a[u] = *(const bf16x8_t *)(H + (p * NO + n) * SW + boff);
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb)
                        b[u][cb] = *(const bf16x8_t *)(Xp + (ls * 64 + cb * 16 + n) * SW + boff);
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], b[u][cb], acc[cb], 0, 0, 0);
        }
        // onsite, moments, store (lane holds alpha = 4g + j of column cb*16 + n)
        float e[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int al = 4 * g + j;
            e[j] = (al < NO) ? (float)H_on[(long)gatom * NO + al] : 0.f;
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const long off = ((long)l * 64 + cb * 16 + n) * SW + 4 * g;
            float xp[4] = {0.f, 0.f, 0.f, 0.f};
            if (has_prev && 4 * g < SW) {
                const unsigned long long v = *(const unsigned long long *)(Xp + off);
#pragma unroll
                for (int j = 0; j < 4; ++j) xp[j] = bf16_to_f32((unsigned short)(v >> (16 * j)));
            }
            float xm[4] = {0.f, 0.f, 0.f, 0.f};
            if (LANCZOS && L <= k - 2 && 4 * g < SW) {
                const unsigned long long v = *(const unsigned long long *)(Xc + off);
#pragma unroll
                for (int j = 0; j < 4; ++j) xm[j] = bf16_to_f32((unsigned short)(v >> (16 * j)));
            }
            unsigned long long outv = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float v = fmaf(e[j], xp[j], acc[cb][j]);
                if (LANCZOS) v = v * ls[cb] - lbeta[cb] * xm[j];
                so[cb] = fma((double)xp[j], (double)v, so[cb]);
                if (!LANCZOS || fin) se[cb] = fma((double)v, (double)v, se[cb]);
                if (LANCZOS && fin) sx[cb] = fma((double)xp[j], (double)xp[j], sx[cb]);
                outv |= (unsigned long long)f32_to_bf16(v) << (16 * j);
            }
            if (keep && 4 * g < SW) *(unsigned long long *)(Xc + off) = outv;
        }
    }
    // sum over the four alpha groups, then over wavefronts in a fixed order
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        so[cb] += __shfl_xor(so[cb], 16); so[cb] += __shfl_xor(so[cb], 32);
        se[cb] += __shfl_xor(se[cb], 16); se[cb] += __shfl_xor(se[cb], 32);
        if constexpr (LANCZOS) { sx[cb] += __shfl_xor(sx[cb], 16); sx[cb] += __shfl_xor(sx[cb], 32); }
    }
    if (g == 0) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            s_red[0][w][cb * 16 + n] = so[cb];
            s_red[1][w][cb * 16 + n] = se[cb];
            if constexpr (LANCZOS) s_red[2][w][cb * 16 + n] = sx[cb];
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        double to = 0.0, te = 0.0, tx = 0.0;
#pragma unroll
        for (int q2 = 0; q2 < NW; ++q2) {
            to += s_red[0][q2][threadIdx.x];
            te += s_red[1][q2][threadIdx.x];
            if constexpr (LANCZOS) tx += s_red[2][q2][threadIdx.x];
        }
        const int ns = LANCZOS && fin ? 3 : 2;
        double *pp = part + (((size_t)t * nch + chunk) * ns) * 64;
        pp[threadIdx.x] = to;
        pp[64 + threadIdx.x] = te;
        if (LANCZOS && fin) pp[128 + threadIdx.x] = tx;
    }
}

// BF16 (or FP16) Lanczos form of the d band on MFMA, one fused pass per
// level (the scheme of k_step with LANCZOS = 1).  Rows are packed without
// padding, two orbitals per 32-bit word, 160 words (640 bytes) per row:
//   W0[c] = (x_0, x_1), W1[c] = (x_2, x_3) of column c (64 words each),
//   W2[c'] = (x_4 of column c', x_4 of column c' + 32), c' < 32.
// A loaded (W0, W1) pair of a column is the B operand of
// v_mfma_f32_16x16x16_bf16 (or _f16) as it stands.  Per row and 16-column block u, the
// K dimension runs over (slot, b): four steps of four slots with b = 0..3
// (lane group g takes slot 4q + g) and one step with b = 4 over slots 4g + i.
// A = the blocks' rows (lane c < 5 of group g reads row c of its slot's
// block from the wave's LDS copy of the row's blocks, the rest are zero;
// the FP16 form reads the FP32 packed blocks and rounds them to FP16 there),
// D[a][16u + c] in lane (c, g) for a = 4g + r.  So a gathered row costs three
// 32-bit loads per column where FP32 costs five, and the level's VMEM
// requests drop by about 40%; the products leave the VALU.  Needs deg_max <=
// 16 (the five K steps cover 16 slots).
constexpr int PK_ROW = 160;
typedef short s16x4_t __attribute__((ext_vector_type(4)));

__device__ inline s16x4_t words_to_s16x4(unsigned lo, unsigned hi)
{
    typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(s16x4_t, (u32x2_t){lo, hi});
}
// the two 16-bit formats of the packed rows: halves of a word to FP32, two
// FP32 values rounded (nearest even) into a word (v_cvt_pk_bf16_f32,
// v_cvt_pk_f16_f32), the 16x16x16 MFMA of the format, and 1.0
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef _Float16 f16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
template <bool F16> struct Half16;
template <> struct Half16<false> {
    static __device__ float lo(unsigned w) { return __uint_as_float(w << 16); }
    static __device__ float hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }
    static __device__ unsigned pack(float a, float b)
    {
        return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
    }
    static __device__ f32x4_t mfma(s16x4_t a, s16x4_t b, f32x4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
    static constexpr unsigned one = 0x3f80u;
};
template <> struct Half16<true> {
    static __device__ float lo(unsigned w) { return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu)); }
    static __device__ float hi(unsigned w) { return (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16)); }
    static __device__ unsigned pack(float a, float b)
    {
        return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2_t){a, b}, f16x2_t));
    }
    static __device__ f32x4_t mfma(s16x4_t a, s16x4_t b, f32x4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(f16x4_t, a), __builtin_bit_cast(f16x4_t, b), c,
                                                     0, 0, 0);
    }
    static constexpr unsigned one = 0x3c00u;
};

template <int WGT, bool F16>
__global__ void __launch_bounds__(WGT)
k_lstep16(Batch bt, int k, int K, int last, int keep, int nch, int chunk_rows, int deg_max, int rows_cap,
          const int *__restrict__ row_ptr, const double *__restrict__ H_on, const void *__restrict__ Hv,
          const int *__restrict__ sizes_, const char *tiles_base, size_t tile_stride, char *xbase,
          size_t x_stride, double *__restrict__ part, const double *__restrict__ lc)
{
    constexpr int NW = WGT / 64, NO = 5, SW = 8;
    using HF = Half16<F16>;
    // a pair's block as stored: BF16 rows padded to 8 ([5][8], 80 bytes), or
    // FP32 packed symmetric (16 values, 64 bytes) for the FP16 vectors
    constexpr int HB = F16 ? BOP_D_PACKED * 4 : NO * SW * 2;
    const char *H = (const char *)Hv;
    __shared__ double s_red[3][NW][64];
    __shared__ __align__(16) float s_d[NW][64 * 8];
    __shared__ __align__(16) char s_h[NW][16 * HB];   // a row's blocks (<= 16 pairs)
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int t = (q / nch) * 8 + xcd, chunk = q % nch;
    if (t >= bt.count) return;
    const int tile = bt.first + t;
    const int *sizes = sizes_ + tile * (MAXK + 2);
    if (sizes[0] < 0) return;
    const int nrow = last ? sizes[K] : sizes[k];
    const int nct = tile_chunks(nrow, chunk_rows, NW);
    if (chunk >= nct) return;
    const int RS = nct * NW;
    const int *sup = (const int *)(tiles_base + tile_stride * tile);
    const int *rinfo = sup + rows_cap;
    const int *lnb = rinfo + rows_cap;
    const int src = last ? (K & 1) : ((k - 1) & 1);
    const unsigned *Xp = (const unsigned *)(xbase + x_stride * (4 * (size_t)t + src));
    unsigned *Xc = (unsigned *)(xbase + x_stride * (4 * (size_t)t + (k & 1)));
    unsigned *Ra = (unsigned *)(xbase + x_stride * (4 * (size_t)t + 2 + ((k - 1) & 1)));
    const unsigned *Rb = (const unsigned *)(xbase + x_stride * (4 * (size_t)t + 2 + (k & 1)));
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *sD = &s_d[w][0];
    char *sH = &s_h[w][0];
    // the lane's column (lane = column in the update): its coefficients, and
    // its own onsite level E_col, by which its chain is shifted (H - E_col
    // leaves the vectors unchanged, a_j comes back shifted), which keeps the
    // BF16 rounding of the stored y' from entering H r_(j-1) with the weight
    // of the onsite level
    const double *lcol = lc + (size_t)t * LC_N * 64 + lane;
    const float ls = (float)lcol[0], lbeta = (float)lcol[64], lcj = (float)lcol[128], lbp = (float)lcol[192],
                linv = (float)lcol[256];
    const int Bt = sizes[0];
    const float ecol = lane < Bt * NO ? (float)H_on[(long)sup[lane / NO] * NO + lane % NO] : 0.f;
    double so = 0.0, se = 0.0, sx = 0.0;
    int l = chunk * NW + w;
    int g_n = 0, info_n = 0, slots_n = 0, p0_n = 0, p1_n = 0;
    // a row's blocks (pairs p0 .. p1, contiguous, 80 bytes each) reach the
    // wave's LDS slice asynchronously (global_load_lds, 16 bytes per lane),
    // issued one row ahead, so the A operands wait for no memory round trip
    if (l < nrow) {
        g_n = cst(sup)[l];
        info_n = cst(rinfo)[l];
        slots_n = lane < deg_max ? lnb[(long)l * deg_max + lane] : 0;
        p0_n = cst(row_ptr)[g_n];
        p1_n = cst(row_ptr)[g_n + 1];
        h_to_lds16((const float *)(H + (long)p0_n * HB), (float *)sH, (p1_n - p0_n) * HB / 4, lane);
    }
    for (; l < nrow; l += RS) {
        const int gatom = g_n, info = info_n, slots_all = slots_n;
        if (l + RS < nrow) {
            g_n = cst(sup)[l + RS];
            info_n = cst(rinfo)[l + RS];
            slots_n = lane < deg_max ? lnb[(long)(l + RS) * deg_max + lane] : 0;
            p0_n = cst(row_ptr)[g_n];
            p1_n = cst(row_ptr)[g_n + 1];
        }
        const int L = info & 255, n1 = (info >> 8) & 255, n2 = (info >> 16) & 255, n3 = (info >> 24) & 255;
        const bool has_prev = last || L <= k - 1;
        const int nval = last ? n3 : (k - 1 >= L + 1 ? n3 : (k - 1 == L ? n2 : n1));
        const int slots = lane < nval ? slots_all : 0;
        // the row's own y'_j, r_(j-1), r_(j-2) (zero outside their supports), one
        // column per lane, issued with the gathers so that the update after the
        // products waits for no further round trip
        const bool h1 = L <= k - 2, h2 = L <= k - 3;
        const long ro = (long)l * PK_ROW;
        const int w2 = 128 + (lane & 31);
        const unsigned x01 = has_prev ? Xp[ro + lane] : 0u, x23 = has_prev ? Xp[ro + 64 + lane] : 0u;
        const unsigned x4w = has_prev ? Xp[ro + w2] : 0u;
        // r is read once: non-temporal loads keep it from displacing gathered rows in L2
        const unsigned p01 = h1 ? __builtin_nontemporal_load(&Rb[ro + lane]) : 0u;
        const unsigned p23 = h1 ? __builtin_nontemporal_load(&Rb[ro + 64 + lane]) : 0u;
        const unsigned p4w = h1 ? __builtin_nontemporal_load(&Rb[ro + w2]) : 0u;
        const unsigned q01 = h2 ? __builtin_nontemporal_load(&Ra[ro + lane]) : 0u;
        const unsigned q23 = h2 ? __builtin_nontemporal_load(&Ra[ro + 64 + lane]) : 0u;
        const unsigned q4w = h2 ? __builtin_nontemporal_load(&Ra[ro + w2]) : 0u;
        // the B operands of the four b = 0..3 steps and the b = 4 step, all
        // loads issued before the first product
        int pkq[4], pki[4];
        unsigned B0[4][4], B1[4][4];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int sl = 4 * qq + g;
            pkq[qq] = __shfl(slots, sl);
#pragma unroll
            for (int u = 0; u < 4; ++u) B0[qq][u] = B1[qq][u] = 0u;
            if (sl < nval) {
                const unsigned *xr = Xp + (long)(pkq[qq] >> 8) * PK_ROW;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    B0[qq][u] = xr[16 * u + c];
                    B1[qq][u] = xr[64 + 16 * u + c];
                }
            }
        }
        unsigned w2a[4], w2b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int sl = 4 * g + i;
            pki[i] = __shfl(slots, sl);
            w2a[i] = w2b[i] = 0u;
            if (sl < nval) {
                const unsigned *xr = Xp + (long)(pki[i] >> 8) * PK_ROW + 128;
                w2a[i] = xr[c];
                w2b[i] = xr[16 + c];
            }
        }
        // this row's blocks have reached LDS (the copy was issued a row ahead):
        // the A operands, lane c < 5 of group g takes row c of its slot's block
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        s16x4_t A[4];
        unsigned short a4[4];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            A[qq] = s16x4_t{0, 0, 0, 0};
            if (4 * qq + g < nval && c < NO) {
                const char *hb = sH + (pkq[qq] & 255) * HB;
                if constexpr (F16) {
                    const float *h = (const float *)hb;
                    A[qq] = words_to_s16x4(HF::pack(h[d_packed_index(c, 0)], h[d_packed_index(c, 1)]),
                                           HF::pack(h[d_packed_index(c, 2)], h[d_packed_index(c, 3)]));
                } else {
                    A[qq] = *(const s16x4_t *)((const unsigned short *)hb + c * SW);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a4[i] = 0;
            if (4 * g + i < nval && c < NO) {
                const char *hb = sH + (pki[i] & 255) * HB;
                if constexpr (F16) a4[i] = (unsigned short)(HF::pack(((const float *)hb)[d_packed_index(c, 4)], 0.f) & 0xffffu);
                else a4[i] = ((const unsigned short *)hb)[c * SW + 4];
            }
        }
        // the next row's blocks into the slice once these reads are done
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        if (l + RS < nrow)
            h_to_lds16((const float *)(H + (long)p0_n * HB), (float *)sH, (p1_n - p0_n) * HB / 4, lane);
        f32x4_t acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            if (4 * qq >= nval) break;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                acc[u] = HF::mfma(A[qq], words_to_s16x4(B0[qq][u], B1[qq][u]), acc[u]);
        }
        if (nval > 0) {
            const s16x4_t A4 = words_to_s16x4((unsigned)a4[0] | ((unsigned)a4[1] << 16),
                                              (unsigned)a4[2] | ((unsigned)a4[3] << 16));
            // x_4 of columns c (low halves) and c + 32 (high halves) of W2[c],
            // of columns 16 + c and 48 + c of W2[16 + c]
            const unsigned lo_a01 = (w2a[0] & 0xffffu) | (w2a[1] << 16), lo_a23 = (w2a[2] & 0xffffu) | (w2a[3] << 16);
            const unsigned hi_a01 = (w2a[0] >> 16) | (w2a[1] & 0xffff0000u),
                           hi_a23 = (w2a[2] >> 16) | (w2a[3] & 0xffff0000u);
            const unsigned lo_b01 = (w2b[0] & 0xffffu) | (w2b[1] << 16), lo_b23 = (w2b[2] & 0xffffu) | (w2b[3] << 16);
            const unsigned hi_b01 = (w2b[0] >> 16) | (w2b[1] & 0xffff0000u),
                           hi_b23 = (w2b[2] >> 16) | (w2b[3] & 0xffff0000u);
            acc[0] = HF::mfma(A4, words_to_s16x4(lo_a01, lo_a23), acc[0]);
            acc[1] = HF::mfma(A4, words_to_s16x4(lo_b01, lo_b23), acc[1]);
            acc[2] = HF::mfma(A4, words_to_s16x4(hi_a01, hi_a23), acc[2]);
            acc[3] = HF::mfma(A4, words_to_s16x4(hi_b01, hi_b23), acc[3]);
        }
        // D to the wave's LDS block as [column][8] (lane (c, g) holds a = 4g..4g+3
        // of column 16u + c), then one column per lane for the update
        __builtin_amdgcn_wave_barrier();
        if (g < 2) {
#pragma unroll
            for (int u = 0; u < 4; ++u) *(f32x4_t *)&sD[(16 * u + c) * 8 + 4 * g] = acc[u];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0xc07f);          // the block's LDS writes are done
        __builtin_amdgcn_wave_barrier();
        const f32x4_t d03 = *(const f32x4_t *)&sD[lane * 8];
        const float d4 = sD[lane * 8 + 4];
        // H y'_j = D + (E - E_col) y'_j, H r_(j-1) = (y'_j + beta_(j-1) r_(j-2)) /
        // s_(j-1), then r_j and y'_(j+1) as in the FP32 form, rounded to BF16
        // when stored; the sums use the stored values
        const bool upper = lane >= 32;
        const float xs[5] = {HF::lo(x01), HF::hi(x01), HF::lo(x23), HF::hi(x23),
                             upper ? HF::hi(x4w) : HF::lo(x4w)};
        const float r1[5] = {HF::lo(p01), HF::hi(p01), HF::lo(p23), HF::hi(p23),
                             upper ? HF::hi(p4w) : HF::lo(p4w)};
        const float r2[5] = {HF::lo(q01), HF::hi(q01), HF::lo(q23), HF::hi(q23),
                             upper ? HF::hi(q4w) : HF::lo(q4w)};
        const float dv[5] = {d03[0], d03[1], d03[2], d03[3], d4};
        float rj[5], y[5];
#pragma unroll
        for (int a = 0; a < NO; ++a) {
            const float hx = fmaf((float)cst(H_on)[(long)gatom * NO + a] - ecol, xs[a], dv[a]);
            const float hrp = (xs[a] + lbp * r2[a]) * linv;
            const float hr = hx - lcj * hrp;
            rj[a] = xs[a] - lcj * r1[a];
            y[a] = ls * hr - lbeta * r1[a];
        }
        // x_4 of column c' + 32 to lane c' for the shared W2 words
        const float rj4u = __shfl_xor(rj[4], 32), y4u = __shfl_xor(y[4], 32);
        const unsigned rw01 = HF::pack(rj[0], rj[1]), rw23 = HF::pack(rj[2], rj[3]);
        const unsigned yw01 = HF::pack(y[0], y[1]), yw23 = HF::pack(y[2], y[3]);
        const unsigned rw4 = upper ? HF::pack(rj4u, rj[4]) : HF::pack(rj[4], rj4u);
        const unsigned yw4 = upper ? HF::pack(y4u, y[4]) : HF::pack(y[4], y4u);
        const float rs[5] = {HF::lo(rw01), HF::hi(rw01), HF::lo(rw23), HF::hi(rw23),
                             upper ? HF::hi(rw4) : HF::lo(rw4)};
        const float ys[5] = {HF::lo(yw01), HF::hi(yw01), HF::lo(yw23), HF::hi(yw23),
                             upper ? HF::hi(yw4) : HF::lo(yw4)};
#pragma unroll
        for (int a = 0; a < NO; ++a) {
            so = fma((double)rs[a], (double)ys[a], so);
            se = fma((double)ys[a], (double)ys[a], se);
            sx = fma((double)rs[a], (double)rs[a], sx);
        }
        // r_j only on the layers later passes read it (not the newest, where it is zero)
        if (keep) {
            if (has_prev) {
                __builtin_nontemporal_store(rw01, &Ra[ro + lane]);
                __builtin_nontemporal_store(rw23, &Ra[ro + 64 + lane]);
            }
            __builtin_nontemporal_store(yw01, &Xc[ro + lane]);
            __builtin_nontemporal_store(yw23, &Xc[ro + 64 + lane]);
            if (!upper) {
                if (has_prev) __builtin_nontemporal_store(rw4, &Ra[ro + w2]);
                __builtin_nontemporal_store(yw4, &Xc[ro + w2]);
            }
        }
    }
    s_red[0][w][lane] = so;
    s_red[1][w][lane] = se;
    s_red[2][w][lane] = sx;
    __syncthreads();
    if (threadIdx.x < 64) {
        double to = 0.0, te = 0.0, tx = 0.0;
#pragma unroll
        for (int q2 = 0; q2 < NW; ++q2) {
            to += s_red[0][q2][threadIdx.x];
            te += s_red[1][q2][threadIdx.x];
            tx += s_red[2][q2][threadIdx.x];
        }
        double *pp = part + (((size_t)t * nch + chunk) * 3) * 64;
        pp[threadIdx.x] = to;
        pp[64 + threadIdx.x] = te;
        pp[128 + threadIdx.x] = tx;
    }
}

// dynamic LDS of a step launch that stages the rows' H blocks (one slice of
// deg_max blocks per wavefront)
static inline size_t h_lds_bytes(const bop_plan &p, int wgt, size_t elem)
{
    return (size_t)(wgt / 64) * h_slice(p.deg_max, p.n_orb == 5 ? BOP_D_PACKED : p.n_orb * p.n_orb) * elem;
}

// static LDS of k_step (its per-wave partial sums), which the H slices share
// the workgroup's LDS with
static inline size_t step_static_lds(int wgt, int lanczos) { return (size_t)(lanczos ? 3 : 2) * wgt * 8; }

template <int NO>
int run_moments_bf16(const bop_plan &p, const int *row_ptr, const double *H_on, const void *Hv, double *mu,
                     char *ws, const Layout &lay, hipStream_t st)
{
    const unsigned short *H = (const unsigned short *)Hv;
    const int K = p.n_max / 2;
    const int steps = K + (p.n_max & 1);
    const int *sizes = (const int *)(ws + lay.sizes);
    const char *tiles = ws + lay.tiles;
    char *xb = ws + lay.x;
    double *part = (double *)(ws + lay.part);
    const StepParts sp = step_parts(p);
    for (int first = 0; first < p.n_tiles; first += p.batch_tiles) {
        Batch bt{first, min(p.batch_tiles, p.n_tiles - first)};
        k_x0_bf16<NO><<<bt.count, 256, 0, st>>>(bt, p.n_max, sizes, tiles, lay.tile_stride, xb, lay.x_stride, mu);
        BOP_LAUNCHED();
        const int nb8 = (bt.count + 7) / 8;
        for (int k = 1; k <= steps; ++k) {
            const int last = k > K;
            // X^K is read again only by the extra step of an odd n_max; for an
            // even n_max its moments come from this step's partial sums
            const int keep = !last && (k < K || (p.n_max & 1));
            const int rows_k = last ? p.rows_k[K] : p.rows_k[k];
            const int nch = (rows_k + p.chunk_rows - 1) / p.chunk_rows;
            if (nch <= 0) continue;
            dim3 grid((unsigned)(nb8 * nch * 8));
#define BOP_STEP16(W)                                                                                    \
    k_step_bf16<NO, W, 0><<<grid, W, 0, st>>>(bt, k, K, last, keep, 0, nch, p.chunk_rows, p.deg_max,          \
                                              p.rows_cap,                                                    \
                                              row_ptr, H_on, H, sizes, tiles, lay.tile_stride, xb, lay.x_stride, \
                                              part + sp.off[k], nullptr)
            if (p.block_threads == 256) BOP_STEP16(256);
            else if (p.block_threads == 512) BOP_STEP16(512);
            else BOP_STEP16(1024);
#undef BOP_STEP16
            BOP_LAUNCHED();
        }
        if (steps > 0) {
            k_reduce<NO><<<dim3((unsigned)bt.count, (unsigned)steps), 64, 0, st>>>(
                bt, K, p.n_max, sp, p.chunk_rows, p.block_threads / 64, sizes, tiles, lay.tile_stride, part, mu);
            BOP_LAUNCHED();
        }
    }
    return BOP_OK;
}

template <typename T, int NO>
int run_moments(const bop_plan &p, const int *row_ptr, const double *H_on, const void *Hv, double *mu,
                char *ws, const Layout &lay, hipStream_t st)
{
    const T *H = (const T *)Hv;
    const int K = p.n_max / 2;
    const int steps = K + (p.n_max & 1);
    const int *sizes = (const int *)(ws + lay.sizes);
    const char *tiles = ws + lay.tiles;
    char *xb = ws + lay.x;
    double *part = (double *)(ws + lay.part);
    const StepParts sp = step_parts(p);
    const size_t lds_max = (size_t)device_lds_per_block();
    for (int first = 0; first < p.n_tiles; first += p.batch_tiles) {
        Batch bt{first, min(p.batch_tiles, p.n_tiles - first)};
        k_x0<T, NO><<<bt.count, 256, 0, st>>>(bt, p.n_max, p.tile_atoms, sizes, tiles, lay.tile_stride, xb,
                                              lay.x_stride, mu);
        BOP_LAUNCHED();
        const int nb8 = (bt.count + 7) / 8;
        for (int k = 1; k <= steps; ++k) {
            const int last = k > K;
            // X^K is read again only by the extra step of an odd n_max; for an
            // even n_max its moments come from this step's partial sums
            const int keep = !last && (k < K || (p.n_max & 1));
            const int rows_k = last ? p.rows_k[K] : p.rows_k[k];
            const int nch = (rows_k + p.chunk_rows - 1) / p.chunk_rows;
            if (nch <= 0) continue;
            dim3 grid((unsigned)(nb8 * nch * 8));
#define BOP_STEP_ARGS                                                                                 \
    bt, k, K, last, keep, 0, nch, p.chunk_rows, p.deg_max, p.rows_cap, row_ptr, H_on, H, sizes, tiles,  \
        lay.tile_stride, xb, lay.x_stride, part + sp.off[k], nullptr
#define BOP_STEP_TR(W, TR)                                                                            \
    do {                                                                                              \
        const size_t lds = h_lds_bytes(p, W, sizeof(T));                                              \
        if constexpr (sizeof(T) == 8) {                                                               \
            k_step<T, NO, W, 0, T, true, TR><<<grid, W, 0, st>>>(BOP_STEP_ARGS);                      \
        } else {                                                                                      \
            if (lds + step_static_lds(W, 0) > lds_max)                                                \
                k_step<T, NO, W, 0, T, true, TR><<<grid, W, 0, st>>>(BOP_STEP_ARGS);                  \
            else k_step<T, NO, W, 0, T, false, TR><<<grid, W, lds, st>>>(BOP_STEP_ARGS);              \
        }                                                                                             \
    } while (0)
#define BOP_STEP(W)                                                                                   \
    do {                                                                                              \
        if (p.r_max > 0.0) BOP_STEP_TR(W, true);                                                      \
        else BOP_STEP_TR(W, false);                                                                   \
    } while (0)
            if (p.block_threads == 256) BOP_STEP(256);
            else if (p.block_threads == 512) BOP_STEP(512);
            else BOP_STEP(1024);
#undef BOP_STEP
#undef BOP_STEP_TR
#undef BOP_STEP_ARGS
            BOP_LAUNCHED();
        }
        if (steps > 0) {
            k_reduce<NO><<<dim3((unsigned)bt.count, (unsigned)steps), 64, 0, st>>>(
                bt, K, p.n_max, sp, p.chunk_rows, p.block_threads / 64, sizes, tiles, lay.tile_stride, part, mu);
            BOP_LAUNCHED();
        }
    }
    return BOP_OK;
}

// ---------------------------------------------------------------------------
// Lanczos form: the recursion coefficients straight from the H.X products
// ---------------------------------------------------------------------------
// The chain of App. B.3 is built column by column with the Lanczos algorithm
// (u_0 = unit start vector, b_(k+1) u_(k+1) = H u_k - a_k u_k - b_k u_(k-1),
// a_k = <u_k, H u_k>), which gives the same a_n, b_n as the moments but keeps
// the vectors orthonormal, so rounding of the stored vectors in FP32 or BF16
// perturbs a_n, b_n by about the unit roundoff times |H| instead of being
// amplified by the ill-conditioned moments-to-coefficients map.  Vectors are
// stored unnormalised (r_k = |r_k| u_k) and scaled by the per-column factor
// when read, so a level costs one product pass, one elementwise update pass and
// two per-column reductions.  The last level of an even n_max needs only b_K, the
// norm of r_K: its product pass also sums |y'|^2 and |r_(K-1)|^2, which give
// |r_K|^2 = |y'|^2 - 2 a^2 + a^2 s^2 |r_(K-1)|^2 with a = <u_(K-1), y'>, so that
// level has no update pass and stores no vector.
//
// Column coefficients lc[t][.][c]: [0] s_k = 1/|r_k|, [1] beta_k = b_k s_(k-1),
// [2] a_k s_k, [3] s_(k-1).

// unit start vectors, coefficients of level 0, b_0 = 0 and flags; NaN
// coefficients for the seeds of failed tiles
template <typename T, int NO, typename S = T>
__global__ void k_l0(Batch bt, int n_max, const int *__restrict__ sizes_, const char *tiles_base,
                     size_t tile_stride, char *xbase, size_t x_stride, int nbuf, double *__restrict__ lc,
                     double *__restrict__ a, double *__restrict__ b, int *__restrict__ flags, int bf16)
{
    const int t = blockIdx.x;
    if (t >= bt.count) return;
    const int tile = bt.first + t;
    const int *sizes = sizes_ + tile * (MAXK + 2);
    const int *sup = (const int *)(tiles_base + tile_stride * tile);
    const int na = n_max >= 1 ? (n_max - 1) / 2 + 1 : 0, nb = n_max / 2;
    const int Bt = sizes[0] < 0 ? sizes[1] : sizes[0];
    const bool failed = sizes[0] < 0;
    for (int e = threadIdx.x; e < Bt * NO; e += blockDim.x) {
        const long gr = (long)sup[e / NO] * NO + e % NO;
        for (int j = 0; j < na; ++j) a[gr * na + j] = failed ? __builtin_nan("") : 0.0;
        for (int j = 0; j <= nb; ++j) b[gr * (nb + 1) + j] = (failed && j > 0) ? __builtin_nan("") : 0.0;
        flags[gr] = failed ? BOP_FLAG_NONFINITE : 0;
    }
    if (failed) return;
    if (threadIdx.x < 64) {
        double *l = lc + (size_t)t * LC_N * 64;
        l[threadIdx.x] = threadIdx.x < Bt * NO ? 1.0 : 0.0;
        for (int q = 1; q < LC_N; ++q) l[q * 64 + threadIdx.x] = 0.0;
    }
    if (bf16 >= 2) {
        // packed 16-bit rows of the d band (2: BF16, 3: FP16): words (x_0, x_1),
        // (x_2, x_3) per column, then (x_4 of c', x_4 of c' + 32)
        const unsigned one = bf16 == 3 ? Half16<true>::one : Half16<false>::one;
        unsigned *X0 = (unsigned *)(xbase + x_stride * ((size_t)nbuf * t));
        for (int e = threadIdx.x; e < Bt * PK_ROW; e += blockDim.x) {
            const int l = e / PK_ROW, wd = e % PK_ROW;
            int c0, a0, c1, a1;
            if (wd < 128) { c0 = c1 = wd & 63; a0 = 2 * (wd >> 6); a1 = a0 + 1; }
            else { c0 = wd - 128; c1 = c0 + 32; a0 = a1 = 4; }
            const unsigned lo = c0 == l * NO + a0 ? one : 0u, hi = c1 == l * NO + a1 ? one : 0u;
            X0[e] = lo | (hi << 16);
        }
    } else if (bf16) {
        constexpr int SW = NO <= 8 ? 8 : 16;
        unsigned short *X0 = (unsigned short *)(xbase + x_stride * ((size_t)nbuf * t));
        for (int e = threadIdx.x; e < Bt * 64 * SW; e += blockDim.x) {
            int l = e / (64 * SW), rest = e % (64 * SW), c = rest / SW, al = rest % SW;
            X0[e] = (al < NO && c == l * NO + al) ? (unsigned short)0x3f80 : (unsigned short)0;
        }
    } else {
        S *X0 = (S *)(xbase + x_stride * ((size_t)nbuf * t));
        for (int e = threadIdx.x; e < Bt * NO * 64; e += blockDim.x) {
            int l = e / (NO * 64), rest = e % (NO * 64), al = rest / 64, c = rest % 64;
            X0[(long)l * NO * 64 + al * 64 + c] = (c == l * NO + al) ? S(1) : S(0);
        }
    }
}

// BF16 Lanczos update (the MFMA form keeps the two-pass scheme): r_k = y' -
// a_(k-1) s_(k-1) r_(k-1) on the rows of the support of X^k (k is the
// moment-step index, level k - 1), in place of y'; partial sums of |r_k|^2 (of
// r_k rounded to BF16, also when keep = 0 leaves y' in place because no later
// level reads r_k).  A thread owns one column of a row: the slot-width vector
// in the BF16 [64][slot width] layout.
template <int NO, int WGT>
__global__ void __launch_bounds__(WGT)
k_lupdate_bf16(Batch bt, int k, int keep, int nch, int chunk_rows, int rows_cap, const int *__restrict__ sizes_,
               const char *tiles_base, size_t tile_stride, char *xbase, size_t x_stride,
               const double *__restrict__ lc, double *__restrict__ part)
{
    constexpr int NW = WGT / 64;
    constexpr int SW = NO <= 8 ? 8 : 16;
    __shared__ double s_red[NW][64];
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
    const int t = (q / nch) * 8 + xcd, chunk = q % nch;
    if (t >= bt.count) return;
    const int tile = bt.first + t;
    const int *sizes = sizes_ + tile * (MAXK + 2);
    if (sizes[0] < 0) return;
    const int nrow = sizes[k];
    const int nct = tile_chunks(nrow, chunk_rows, NW);
    if (chunk >= nct) return;
    const int *sup = (const int *)(tiles_base + tile_stride * tile);
    const int *rinfo = sup + rows_cap;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int src = (k - 1) & 1, dst = k & 1;
    const double as = lc[((size_t)t * LC_N + 2) * 64 + lane];
    double se = 0.0;
    const unsigned short *Xp = (const unsigned short *)(xbase + x_stride * (2 * (size_t)t + src));
    unsigned short *Xc = (unsigned short *)(xbase + x_stride * (2 * (size_t)t + dst));
    const float asf = (float)as;
    for (int l = chunk * NW + w; l < nrow; l += nct * NW) {
        const bool hp = (rinfo[l] & 255) <= k - 1;
        const long off = ((long)l * 64 + lane) * SW;
#pragma unroll
        for (int al = 0; al < NO; ++al) {
            const float y = bf16_to_f32(Xc[off + al]);
            const float x = hp ? bf16_to_f32(Xp[off + al]) : 0.f;
            const float r = fmaf(-asf, x, y);
            const unsigned short rb = f32_to_bf16(r);
            if (keep) Xc[off + al] = rb;
            const double rd = (double)bf16_to_f32(rb);
            se = fma(rd, rd, se);
        }
    }
    s_red[w][lane] = se;
    __syncthreads();
    if (threadIdx.x < 64) {
        double tot = 0.0;
#pragma unroll
        for (int q2 = 0; q2 < NW; ++q2) tot += s_red[q2][threadIdx.x];
        part[(((size_t)t * nch + chunk) * 2 + 1) * 64 + threadIdx.x] = tot;
    }
}

// Sum of one partial slot over a tile's chunks, in chunk order, eight chunks'
// loads in flight.
__device__ inline double chunk_sum(const double *part, int t, int nch, int used, int ns, int slot, int c)
{
    double sum = 0.0;
    for (int q0 = 0; q0 < used; q0 += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(((size_t)t * nch + min(q0 + u, used - 1)) * ns + slot) * 64 + c];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (q0 + u < used) sum += v[u];
    }
    return sum;
}

// Per-column reduction of level k - 1 of the BF16 two-pass scheme, in chunk
// order.  which = 0: a_(k-1) from the product pass (slot 0); which = 1: b_k from
// the update pass (slot 1), with the breakdown test of the moment route (b_k^2
// <= thr * b_1^2 ends the chain, later a repeat the last one and later b are
// zero); which = 2: both, from the three partials of a last product pass
// (<r_(k-1), y'>, |y'|^2, |r_(k-1)|^2).
__global__ void k_lreduce(Batch bt, int k, int K, int last, int which, int n_max, int no, int nch,
                          int chunk_rows, int nw, double thr, const int *__restrict__ sizes_, const char *tiles_base,
                          size_t tile_stride, const double *__restrict__ part, double *__restrict__ lc,
                          double *__restrict__ a, double *__restrict__ b, int *__restrict__ flags)
{
    const int t = blockIdx.x;
    if (t >= bt.count) return;
    const int tile = bt.first + t;
    const int *sizes = sizes_ + tile * (MAXK + 2);
    if (sizes[0] < 0) return;
    const int c = threadIdx.x;
    if (c >= sizes[0] * no) return;
    const int nrow = last ? sizes[K] : sizes[k];
    const int used = tile_chunks(nrow, chunk_rows, nw);
    const int ns = which == 2 ? 3 : 2;
    double sum = chunk_sum(part, t, nch, used, ns, which == 1 ? 1 : 0, c);
    const int *sup = (const int *)(tiles_base + tile_stride * tile);
    const long gr = (long)sup[c / no] * no + c % no;
    const int na = n_max >= 1 ? (n_max - 1) / 2 + 1 : 0, nb = n_max / 2;
    const int lev = k - 1;
    double *l = lc + (size_t)t * LC_N * 64;
    int fl = flags[gr];
    const bool broke = fl & BOP_FLAG_BREAKDOWN;
    if (!isfinite(sum)) fl |= BOP_FLAG_NONFINITE;
    if (which != 1) {
        const double s = l[c];
        const double av = broke ? a[gr * na + lev - 1] : s * sum;
        a[gr * na + lev] = av;
        l[128 + c] = broke ? 0.0 : av * s;
        if (which == 2) {
            // |r_k|^2 = |y'|^2 - 2 a <u, y'> + a^2 |u|^2 with u = s r_(k-1), <u, y'> = a
            const double yy = chunk_sum(part, t, nch, used, ns, 1, c), xx = chunk_sum(part, t, nch, used, ns, 2, c);
            if (!isfinite(yy) || !isfinite(xx)) fl |= BOP_FLAG_NONFINITE;
            sum = yy - 2.0 * av * av + av * av * s * s * xx;
        }
    }
    if (which != 0) {
        if (!broke) {
            const double var = lev == 0 ? sum : b[gr * (nb + 1) + 1] * b[gr * (nb + 1) + 1];
            if (!(sum > thr * var) || !(sum > 0.0)) {
                for (int j = lev + 1; j <= nb; ++j) b[gr * (nb + 1) + j] = 0.0;
                fl |= BOP_FLAG_BREAKDOWN | ((lev + 1) << 8);
                l[192 + c] = l[c];
                l[c] = 0.0;
                l[64 + c] = 0.0;
            } else {
                const double bb = sqrt(sum);
                b[gr * (nb + 1) + lev + 1] = bb;
                l[192 + c] = l[c];
                l[64 + c] = bb * l[c];
                l[c] = 1.0 / bb;
            }
        }
    }
    flags[gr] = fl;
}

// Per-column reduction after a fused Lanczos pass (level j = k - 1), in chunk
// order: a_j = s_j <r_j, y'_(j+1)>; unless this is the last level of an odd
// n_max, b_(j+1)^2 = |y'_(j+1)|^2 - 2 a_j^2 + a_j^2 s_j^2 |r_j|^2 (the squared
// norm of r_(j+1) = y'_(j+1) - a_j u_j, u_j = s_j r_j; FP64 sums of the stored
// vectors, so its cancellation error is about 1e-16 |y'|^2), with the
// breakdown test of the moment route (b_(j+1)^2 <= thr b_1^2 ends the chain:
// later a repeat the last one, later b are zero and the column's coefficients
// become zero, so its vectors stay zero).  Then the next level's column
// coefficients: s_(j+1) = 1/b_(j+1), beta_(j+1) = b_(j+1) s_j, c_(j+1) = a_j s_j,
// beta_j and 1/s_j.
__global__ void k_lreduce_fused(Batch bt, int k, int K, int last, int n_max, int no, int nch, int chunk_rows,
                                int nw, double thr, const int *__restrict__ sizes_, const char *tiles_base,
                                size_t tile_stride, const double *__restrict__ part, double *__restrict__ lc,
                                double *__restrict__ a, double *__restrict__ b, int *__restrict__ flags,
                                const double *__restrict__ a_shift)
{
    const int t = blockIdx.x;
    if (t >= bt.count) return;
    const int tile = bt.first + t;
    const int *sizes = sizes_ + tile * (MAXK + 2);
    if (sizes[0] < 0) return;
    const int c = threadIdx.x;
    if (c >= sizes[0] * no) return;
    const int nrow = last ? sizes[K] : sizes[k];
    const int used = tile_chunks(nrow, chunk_rows, nw);
    const double ry = chunk_sum(part, t, nch, used, 3, 0, c);
    const double yy = chunk_sum(part, t, nch, used, 3, 1, c);
    const double rr = chunk_sum(part, t, nch, used, 3, 2, c);
    const int *sup = (const int *)(tiles_base + tile_stride * tile);
    const long gr = (long)sup[c / no] * no + c % no;
    const int na = n_max >= 1 ? (n_max - 1) / 2 + 1 : 0, nb = n_max / 2;
    const int lev = k - 1;
    double *l = lc + (size_t)t * LC_N * 64 + c;
    int fl = flags[gr];
    const bool broke = fl & BOP_FLAG_BREAKDOWN;
    if (!isfinite(ry) || !isfinite(yy) || !isfinite(rr)) fl |= BOP_FLAG_NONFINITE;
    const double s = l[0];
    // a_shift: the passes ran on H - a_shift[column] (the coefficients of the
    // shifted chain; a_j gets the shift back)
    const double av = broke ? 0.0 : s * ry;
    a[gr * na + lev] = broke ? a[gr * na + lev - 1] : av + (a_shift ? a_shift[gr] : 0.0);
    if (!last && !broke) {
        const double bsq = yy - 2.0 * av * av + av * av * s * s * rr;
        const double var = lev == 0 ? bsq : b[gr * (nb + 1) + 1] * b[gr * (nb + 1) + 1];
        if (!(bsq > thr * var) || !(bsq > 0.0)) {
            for (int j = lev + 1; j <= nb; ++j) b[gr * (nb + 1) + j] = 0.0;
            fl |= BOP_FLAG_BREAKDOWN | ((lev + 1) << 8);
            for (int q = 0; q < 5; ++q) l[q * 64] = 0.0;
        } else {
            const double bb = sqrt(bsq);
            b[gr * (nb + 1) + lev + 1] = bb;
            l[192] = l[64];                       // beta_j
            l[256] = s > 0.0 ? 1.0 / s : 0.0;     // 1/s_j
            l[64] = bb * s;                       // beta_(j+1)
            l[128] = av * s;                      // c_(j+1)
            l[0] = 1.0 / bb;                      // s_(j+1)
        }
    }
    flags[gr] = fl;
}

// BF16 Lanczos: product pass (k_step_bf16) and update pass per level.
template <int NO>
int run_lanczos_bf16(const bop_plan &p, const int *row_ptr, const double *H_on, const void *Hv, double *a,
                     double *b, int *flags, char *ws, const Layout &lay, hipStream_t st)
{
    const int K = p.n_max / 2;
    const int steps = K + (p.n_max & 1);
    const int *sizes = (const int *)(ws + lay.sizes);
    const char *tiles = ws + lay.tiles;
    char *xb = ws + lay.x;
    double *part = (double *)(ws + lay.part);
    double *lc = (double *)(ws + lay.lc);
    // breakdown threshold on b^2 relative to b_1^2, above the rounding level of the stored vectors
    const double thr = 1e-5;
    for (int first = 0; first < p.n_tiles; first += p.batch_tiles) {
        Batch bt{first, min(p.batch_tiles, p.n_tiles - first)};
        k_l0<float, NO><<<bt.count, 256, 0, st>>>(bt, p.n_max, sizes, tiles, lay.tile_stride, xb, lay.x_stride, 2,
                                                  lc, a, b, flags, 1);
        BOP_LAUNCHED();
        const int nb8 = (bt.count + 7) / 8;
        for (int k = 1; k <= steps; ++k) {
            const int last = k > K;
            const int rows_k = last ? p.rows_k[K] : p.rows_k[k];
            const int nch = (rows_k + p.chunk_rows - 1) / p.chunk_rows;
            if (nch <= 0) continue;
            // the last level of an even n_max: b_K from the product's partials
            // (|r_K|^2 = |y'|^2 - 2 a^2 + a^2 s^2 |r_(K-1)|^2), so y' is not stored
            // and no update pass follows
            const int fin = !last && k == K && !(p.n_max & 1);
            dim3 grid((unsigned)(nb8 * nch * 8));
#define BOP_LSTEP16(W)                                                                                   \
    k_step_bf16<NO, W, 1><<<grid, W, 0, st>>>(bt, k, K, last, !last && !fin, fin, nch, p.chunk_rows,    \
                                              p.deg_max, p.rows_cap, row_ptr, H_on,                      \
                                              (const unsigned short *)Hv, sizes, tiles, lay.tile_stride, \
                                              xb, lay.x_stride, part, lc)
            if (p.block_threads == 256) BOP_LSTEP16(256);
            else if (p.block_threads == 512) BOP_LSTEP16(512);
            else BOP_LSTEP16(1024);
#undef BOP_LSTEP16
            BOP_LAUNCHED();
            k_lreduce<<<bt.count, 64, 0, st>>>(bt, k, K, last, fin ? 2 : 0, p.n_max, NO, nch, p.chunk_rows,
                                               p.block_threads / 64, thr, sizes, tiles, lay.tile_stride, part, lc,
                                               a, b, flags);
            BOP_LAUNCHED();
            if (last || fin) continue;
            // r_K is read again only by the extra level of an odd n_max; for an
            // even n_max only its norm (b_K) is needed
            const int keep = k < K || (p.n_max & 1);
#define BOP_LUPD(W)                                                                                        \
    k_lupdate_bf16<NO, W><<<grid, W, 0, st>>>(bt, k, keep, nch, p.chunk_rows, p.rows_cap, sizes, tiles,    \
                                              lay.tile_stride, xb, lay.x_stride, lc, part)
            if (p.block_threads == 256) BOP_LUPD(256);
            else if (p.block_threads == 512) BOP_LUPD(512);
            else BOP_LUPD(1024);
#undef BOP_LUPD
            BOP_LAUNCHED();
            k_lreduce<<<bt.count, 64, 0, st>>>(bt, k, K, last, 1, p.n_max, NO, nch, p.chunk_rows, p.block_threads / 64,
                                               thr, sizes, tiles, lay.tile_stride, part, lc, a, b, flags);
            BOP_LAUNCHED();
        }
    }
    return BOP_OK;
}

// BF16 Lanczos of the d band on MFMA (k_lstep16): one fused pass per level
// as in the FP32 form, four packed vectors per tile, so a batch holds half
// the plan's tiles in the same X buffers.
template <bool F16>
int run_lanczos16(const bop_plan &p, const int *row_ptr, const double *H_on, const void *Hv, double *a, double *b,
                  int *flags, char *ws, const Layout &lay, hipStream_t st)
{
    const int K = p.n_max / 2;
    const int steps = K + (p.n_max & 1);
    const int *sizes = (const int *)(ws + lay.sizes);
    const char *tiles = ws + lay.tiles;
    char *xb = ws + lay.x;
    double *part = (double *)(ws + lay.part);
    double *lc = (double *)(ws + lay.lc);
    // breakdown threshold on b^2 relative to b_1^2, above the rounding level of the 16-bit vectors
    const double thr = F16 ? 1e-7 : 1e-5;
    const int lbt = p.batch_tiles >= 2 ? p.batch_tiles / 2 : 1;
    for (int first = 0; first < p.n_tiles; first += lbt) {
        Batch bt{first, min(lbt, p.n_tiles - first)};
        k_l0<float, 5><<<bt.count, 256, 0, st>>>(bt, p.n_max, sizes, tiles, lay.tile_stride, xb, lay.x_stride, 4, lc,
                                                 a, b, flags, F16 ? 3 : 2);
        BOP_LAUNCHED();
        const int nb8 = (bt.count + 7) / 8;
        for (int k = 1; k <= steps; ++k) {
            const int last = k > K;
            const int rows_k = last ? p.rows_k[K] : p.rows_k[k];
            const int nch = (rows_k + p.chunk_rows - 1) / p.chunk_rows;
            if (nch <= 0) continue;
            const int keep = k < steps;
            dim3 grid((unsigned)(nb8 * nch * 8));
#define BOP_LSTEP16(W)                                                                                       \
    k_lstep16<W, F16><<<grid, W, 0, st>>>(bt, k, K, last, keep, nch, p.chunk_rows, p.deg_max, p.rows_cap,      \
                                          row_ptr, H_on, Hv, sizes, tiles, lay.tile_stride, xb, lay.x_stride, part, \
                                          lc)
            if (p.block_threads == 256) BOP_LSTEP16(256);
            else if (p.block_threads == 512) BOP_LSTEP16(512);
            else BOP_LSTEP16(1024);
#undef BOP_LSTEP16
            BOP_LAUNCHED();
            k_lreduce_fused<<<bt.count, 64, 0, st>>>(bt, k, K, last, p.n_max, 5, nch, p.chunk_rows,
                                                     p.block_threads / 64, thr, sizes, tiles, lay.tile_stride, part,
                                                     lc, a, b, flags, H_on);
            BOP_LAUNCHED();
        }
    }
    return BOP_OK;
}

// FP64 / FP32 (FP16 vector storage) Lanczos: one fused pass per level (k_step
// with LANCZOS = 1, four vectors per tile, so a batch holds half the plan's
// tiles in the same X buffers) and one column reduction.
template <typename T, int NO, typename S = T>
int run_lanczos(const bop_plan &p, const int *row_ptr, const double *H_on, const void *Hv, double *a, double *b,
                int *flags, char *ws, const Layout &lay, hipStream_t st)
{
    const int K = p.n_max / 2;
    const int steps = K + (p.n_max & 1);
    const int *sizes = (const int *)(ws + lay.sizes);
    const char *tiles = ws + lay.tiles;
    char *xb = ws + lay.x;
    double *part = (double *)(ws + lay.part);
    const size_t lds_max = (size_t)device_lds_per_block();
    double *lc = (double *)(ws + lay.lc);
    // breakdown threshold on b^2 relative to b_1^2, above the rounding level of the stored vectors
    const double thr = p.dtype == BOP_F64 ? 1e-14 : (p.dtype == BOP_F32 ? 1e-10 : 1e-7);
    const int lbt = p.batch_tiles >= 2 ? p.batch_tiles / 2 : 1;
    for (int first = 0; first < p.n_tiles; first += lbt) {
        Batch bt{first, min(lbt, p.n_tiles - first)};
        k_l0<T, NO, S><<<bt.count, 256, 0, st>>>(bt, p.n_max, sizes, tiles, lay.tile_stride, xb, lay.x_stride, 4, lc,
                                                 a, b, flags, 0);
        BOP_LAUNCHED();
        const int nb8 = (bt.count + 7) / 8;
        for (int k = 1; k <= steps; ++k) {
            const int last = k > K;
            const int rows_k = last ? p.rows_k[K] : p.rows_k[k];
            const int nch = (rows_k + p.chunk_rows - 1) / p.chunk_rows;
            if (nch <= 0) continue;
            // the last pass stores nothing: only its partial sums are used
            const int keep = k < steps;
            dim3 grid((unsigned)(nb8 * nch * 8));
#define BOP_LSTEP_ARGS                                                                                \
    bt, k, K, last, keep, 0, nch, p.chunk_rows, p.deg_max, p.rows_cap, row_ptr, H_on, (const T *)Hv,    \
        sizes, tiles, lay.tile_stride, xb, lay.x_stride, part, lc
#define BOP_LSTEP_TR(W, TR)                                                                           \
    do {                                                                                              \
        const size_t lds = h_lds_bytes(p, W, sizeof(T));                                              \
        if constexpr (sizeof(T) == 8) {                                                               \
            k_step<T, NO, W, 1, S, true, TR><<<grid, W, 0, st>>>(BOP_LSTEP_ARGS);                     \
        } else {                                                                                      \
            if (lds + step_static_lds(W, 1) > lds_max)                                                \
                k_step<T, NO, W, 1, S, true, TR><<<grid, W, 0, st>>>(BOP_LSTEP_ARGS);                 \
            else k_step<T, NO, W, 1, S, false, TR><<<grid, W, lds, st>>>(BOP_LSTEP_ARGS);             \
        }                                                                                             \
    } while (0)
#define BOP_LSTEP(W)                                                                                  \
    do {                                                                                              \
        if (p.r_max > 0.0) BOP_LSTEP_TR(W, true);                                                     \
        else BOP_LSTEP_TR(W, false);                                                                  \
    } while (0)
            if (p.block_threads == 256) BOP_LSTEP(256);
            else if (p.block_threads == 512) BOP_LSTEP(512);
            else BOP_LSTEP(1024);
#undef BOP_LSTEP
#undef BOP_LSTEP_TR
#undef BOP_LSTEP_ARGS
            BOP_LAUNCHED();
            k_lreduce_fused<<<bt.count, 64, 0, st>>>(bt, k, K, last, p.n_max, NO, nch, p.chunk_rows,
                                                     p.block_threads / 64, thr, sizes, tiles, lay.tile_stride, part,
                                                     lc, a, b, flags, nullptr);
            BOP_LAUNCHED();
        }
    }
    return BOP_OK;
}

int default_tile_atoms(int no) { return 64 / no; }

}  // namespace
}  // namespace bop

using namespace bop;

// Device form of a path radius; checks that r_max + r_cut is below half the
// smallest cell height (where the minimum image of every atom within r_max is
// unique and the fractional rounding finds it).
static int make_radius(const bop_path_radius *r, Radius *out, const char *who)
{
    *out = Radius{};
    if (!r) return BOP_OK;
    BOP_REQUIRE(r->r_max > 0.0 && r->r_cut >= 0.0 && r->pos, BOP_E_ARG, "%s: path radius needs r_max > 0 and positions",
                who);
    const double *A = r->cell;
    auto cross = [](const double *u, const double *v, double *w) {
        w[0] = u[1] * v[2] - u[2] * v[1];
        w[1] = u[2] * v[0] - u[0] * v[2];
        w[2] = u[0] * v[1] - u[1] * v[0];
    };
    double c23[3], c31[3], c12[3];
    cross(A + 3, A + 6, c23);
    cross(A + 6, A + 0, c31);
    cross(A + 0, A + 3, c12);
    const double V = A[0] * c23[0] + A[1] * c23[1] + A[2] * c23[2];
    BOP_REQUIRE(std::fabs(V) > 0.0, BOP_E_ARG, "%s: singular cell", who);
    const double *cs[3] = {c23, c31, c12};
    double hmin = INFINITY;
    for (int a = 0; a < 3; ++a) {
        const double nrm = std::sqrt(cs[a][0] * cs[a][0] + cs[a][1] * cs[a][1] + cs[a][2] * cs[a][2]);
        hmin = std::fmin(hmin, std::fabs(V) / nrm);
    }
    BOP_REQUIRE(r->r_max + r->r_cut < 0.5 * hmin, BOP_E_ARG,
                "%s: r_max + r_cut = %g must be below half the smallest cell height (%g)", who, r->r_max + r->r_cut,
                0.5 * hmin);
    out->on = 1;
    out->r2 = r->r_max * r->r_max;
    for (int e = 0; e < 9; ++e) out->A[e] = A[e];
    // inverse of the row-vector cell matrix: column a of it is (a_b x a_c) / V
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) out->Ai[b * 3 + a] = cs[a][b] / V;
    out->pos = r->pos;
    return BOP_OK;
}

extern "C" size_t bop_moments_plan_scratch_size(int n_atoms)
{
    if (n_atoms < 0) return 0;
    size_t per = align_up(4ull * n_atoms, 256) * 2;
    return HDR + (size_t)map_workgroups(n_atoms, 1 << 30) * per;
}

extern "C" int bop_moments_plan(int n_atoms, int n_orb, int n_max, int dtype, const int *row_ptr,
                                const int *nbr_j, const int *order, const bop_tuning *tuning,
                                const bop_path_radius *radius, void *scratch, size_t scratch_bytes, bop_plan *plan,
                                hipStream_t stream)
{
    BOP_REQUIRE(plan && n_atoms >= 0, BOP_E_ARG, "bop_moments_plan: bad arguments");
    BOP_REQUIRE(n_orb == 5 || n_orb == 9, BOP_E_UNSUPPORTED, "bop_moments_plan: n_orb must be 5 or 9");
    BOP_REQUIRE(n_max >= 0 && n_max <= MAX_NMAX, BOP_E_UNSUPPORTED, "bop_moments_plan: n_max must be 0..%d", MAX_NMAX);
    BOP_REQUIRE(dtype == BOP_F64 || dtype == BOP_F32 || dtype == BOP_BF16 || dtype == BOP_F16, BOP_E_UNSUPPORTED,
                "bop_moments_plan: unknown dtype %d", dtype);
    BOP_REQUIRE(n_atoms == 0 || (row_ptr && nbr_j), BOP_E_ARG, "bop_moments_plan: neighbour arrays NULL");
    BOP_REQUIRE(!radius || dtype != BOP_BF16, BOP_E_UNSUPPORTED,
                "bop_moments_plan: a path radius is not supported with BF16 H.X");
    Radius rad;
    if (int rc = make_radius(radius, &rad, "bop_moments_plan")) return rc;
    size_t need = bop_moments_plan_scratch_size(n_atoms);
    BOP_REQUIRE(scratch && scratch_bytes >= need, BOP_E_CAPACITY,
                "bop_moments_plan: scratch of %zu bytes needed", need);
    const int B = (tuning && tuning->tile_atoms > 0) ? tuning->tile_atoms : default_tile_atoms(n_orb);
    BOP_REQUIRE(B * n_orb <= 64, BOP_E_UNSUPPORTED, "bop_moments_plan: tile_atoms * n_orb must be <= 64");
    const int wgt = (tuning && tuning->block_threads) ? tuning->block_threads : 512;
    BOP_REQUIRE(wgt == 256 || wgt == 512 || wgt == 1024, BOP_E_UNSUPPORTED,
                "bop_moments_plan: block_threads must be 256, 512 or 1024");
    // rows per workgroup and step: 64; 128 for the 16-bit d band, whose MFMA
    // Lanczos pass is 4% faster with it (its moment form is 1% slower)
    const int chunk = (tuning && tuning->chunk_rows > 0)
                          ? tuning->chunk_rows
                          : ((dtype == BOP_BF16 || dtype == BOP_F16) && n_orb == 5 ? 128 : 64);
    const int n_tiles = (n_atoms + B - 1) / B;
    const int K = n_max / 2;

    int *hdr = (int *)scratch;
    char *base = (char *)scratch + HDR;
    const size_t per = align_up(4ull * n_atoms, 256) * 2;
    const int pwg = map_workgroups(n_atoms, n_tiles > 0 ? n_tiles : 1);
    // one bit per atom in LDS when that fits a workgroup (two per CU)
    const size_t bits_bytes = 4ull * ((n_atoms + 31) / 32);
    const int search = tuning ? tuning->plan_search : 0;
    BOP_REQUIRE(search >= 0 && search <= 2, BOP_E_ARG, "bop_moments_plan: plan_search must be 0, 1 or 2");
    const bool fits = bits_bytes + 16 * 1024 <= (size_t)device_lds_per_block() && bits_bytes <= 64 * 1024;
    BOP_REQUIRE(search != 1 || fits, BOP_E_UNSUPPORTED, "bop_moments_plan: %d atoms too many for the LDS bitmap",
                n_atoms);
    const bool bits = search == 1 || (search == 0 && fits);
    long nmap = bits ? 0 : (long)pwg * (long)(per / 4);
    k_init<<<(unsigned)((nmap + 255) / 256 > 0 ? (nmap + 255) / 256 : 1), 256, 0, stream>>>(hdr, HDR / 4,
                                                                                           (int *)base, nmap);
    BOP_LAUNCHED();
    int hv[HDR / 4] = {};
    if (n_atoms > 0) {
        k_max_degree<<<(n_atoms + 255) / 256, 256, 0, stream>>>(n_atoms, row_ptr, hdr);
        BOP_LAUNCHED();
        BOP_HIP(hipMemcpyAsync(hv, hdr, sizeof hv, hipMemcpyDeviceToHost, stream));
        BOP_HIP(hipStreamSynchronize(stream));
        BOP_REQUIRE(hv[3] <= 64, BOP_E_UNSUPPORTED, "bop_moments_plan: %d neighbours in a row (at most 64)", hv[3]);
        int dmax = hv[3] > 0 ? hv[3] : 1;
        // the breadth-first claims encode (row, slot) entries as CLAIM + entry < 2^31
        BOP_REQUIRE((long)n_atoms * dmax < (1L << 30), BOP_E_UNSUPPORTED,
                    "bop_moments_plan: %d atoms x %d neighbours too large for one plan (split the structure)", n_atoms,
                    dmax);
        if (bits)
            k_plan_bits<<<pwg, PLAN_T, bits_bytes, stream>>>(n_atoms, B, n_tiles, K, order, row_ptr, nbr_j, dmax,
                                                            hdr, base, per, rad);
        else
            k_plan<<<pwg, PLAN_T, 0, stream>>>(n_atoms, B, n_tiles, K, order, row_ptr, nbr_j, dmax, hdr, base, per,
                                               rad);
        BOP_LAUNCHED();
        BOP_HIP(hipMemcpyAsync(hv, hdr, sizeof hv, hipMemcpyDeviceToHost, stream));
        BOP_HIP(hipStreamSynchronize(stream));
    }
    *plan = bop_plan{};
    plan->n_atoms = n_atoms;
    plan->n_orb = n_orb;
    plan->n_max = n_max;
    plan->dtype = dtype;
    plan->tile_atoms = B;
    plan->n_tiles = n_tiles;
    plan->block_threads = wgt;
    plan->chunk_rows = chunk;
    plan->deg_max = hv[3] > 0 ? hv[3] : 1;
    plan->rows_cap = hv[2] > 0 ? hv[2] : 1;
    for (int k = 0; k <= K; ++k) plan->rows_k[k] = hv[8 + k];
    plan->search = bits ? 1 : 2;
    plan->r_max = radius ? radius->r_max : 0.0;
    BOP_REQUIRE(plan->rows_cap < (1 << 23), BOP_E_UNSUPPORTED, "bop_moments_plan: tile support too large");
    const size_t x_tile = 2 * align_up(x_row_bytes(dtype, n_orb) * plan->rows_cap, 256);
    // default batch: 48 GiB of X buffers, at most a quarter of the free device
    // memory (larger batches mean fewer launches and fewer partly idle launch
    // tails: at 128,000 atoms 24 -> 48 GiB took the FP32 Lanczos pass from 220
    // to 216 ms and the FP64 moment pass from 341 to 337 ms)
    size_t x_budget = 48ull << 30, mem_free = 0, mem_total = 0;
    if (hipMemGetInfo(&mem_free, &mem_total) == hipSuccess && mem_free / 4 < x_budget) x_budget = mem_free / 4;
    if (x_budget < (1ull << 30)) x_budget = 1ull << 30;
    long bt = (tuning && tuning->batch_tiles > 0) ? tuning->batch_tiles : (long)(x_budget / x_tile);
    bt = bt < 8 ? 8 : bt;
    bt = (bt / 8) * 8;
    if (bt > n_tiles) bt = n_tiles > 0 ? n_tiles : 1;
    plan->batch_tiles = (int)bt;
    plan->ws_bytes = make_layout(*plan, map_workgroups(n_atoms, n_tiles > 0 ? n_tiles : 1)).bytes;
    return BOP_OK;
}

extern "C" int bop_moments_prepare(const bop_plan *plan, const int *row_ptr, const int *nbr_j, const int *order,
                                   const bop_path_radius *radius, void *ws, size_t ws_bytes, hipStream_t stream)
{
    BOP_REQUIRE(plan, BOP_E_ARG, "bop_moments_prepare: plan is NULL");
    BOP_REQUIRE((plan->r_max > 0.0) == (radius != nullptr) && (!radius || radius->r_max == plan->r_max), BOP_E_ARG,
                "bop_moments_prepare: give the plan's path radius (and none if the plan has none)");
    Radius rad;
    if (int rc = make_radius(radius, &rad, "bop_moments_prepare")) return rc;
    BOP_REQUIRE(ws && ws_bytes >= plan->ws_bytes, BOP_E_CAPACITY,
                "bop_moments_prepare: workspace of %zu bytes needed, %zu given", plan->ws_bytes, ws_bytes);
    const int n = plan->n_atoms;
    if (n == 0) return BOP_OK;
    BOP_REQUIRE(row_ptr && nbr_j, BOP_E_ARG, "bop_moments_prepare: neighbour arrays NULL");
    const int pwg = map_workgroups(n, plan->n_tiles);
    Layout lay = make_layout(*plan, pwg);
    const size_t map_stride = align_up(4ull * n, 256);
    int *hdr = (int *)ws;
    char *w = (char *)ws;
    long nmap = (long)pwg * (long)(map_stride / 4);
    k_init<<<(unsigned)((nmap + 255) / 256), 256, 0, stream>>>(hdr, 8, (int *)(w + lay.x), nmap);
    BOP_LAUNCHED();
    RowsK rk{};
    for (int k = 0; k <= plan->n_max / 2; ++k) rk.r[k] = plan->rows_k[k];
    // the ordered search with two LDS bitmaps where they fit a workgroup
    const size_t bits2 = 2 * 4ull * ((n + 31) / 32);
    const bool bits = plan->search == 1 && bits2 + 16 * 1024 <= (size_t)device_lds_per_block() && bits2 <= 128 * 1024;
    if (bits)
        k_prepare<true><<<pwg, PLAN_T, bits2, stream>>>(n, plan->tile_atoms, plan->n_tiles, plan->n_max / 2, order,
                                                        row_ptr, nbr_j, plan->deg_max, plan->rows_cap, rk, hdr, w,
                                                        lay, map_stride, rad);
    else
        k_prepare<false><<<pwg, PLAN_T, 0, stream>>>(n, plan->tile_atoms, plan->n_tiles, plan->n_max / 2, order,
                                                     row_ptr, nbr_j, plan->deg_max, plan->rows_cap, rk, hdr, w,
                                                     lay, map_stride, rad);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" int bop_moments(const bop_plan *plan, const int *row_ptr, const double *H_on, const void *H_bond,
                           double *mu, void *ws, size_t ws_bytes, hipStream_t stream)
{
    BOP_REQUIRE(plan, BOP_E_ARG, "bop_moments: plan is NULL");
    BOP_REQUIRE(ws && ws_bytes >= plan->ws_bytes, BOP_E_CAPACITY,
                "bop_moments: workspace of %zu bytes needed, %zu given", plan->ws_bytes, ws_bytes);
    const int n = plan->n_atoms, no = plan->n_orb;
    if (n == 0) return BOP_OK;
    BOP_REQUIRE(row_ptr && H_on && H_bond && mu, BOP_E_ARG, "bop_moments: NULL array");
    Layout lay = make_layout(*plan, map_workgroups(n, plan->n_tiles));
    char *w = (char *)ws;
    BOP_REQUIRE(plan->dtype != BOP_F16, BOP_E_UNSUPPORTED,
                "bop_moments: FP16 vector storage is for the Lanczos form (bop_lanczos) only");
    if (plan->dtype == BOP_BF16)
        return no == 5 ? run_moments_bf16<5>(*plan, row_ptr, H_on, H_bond, mu, w, lay, stream)
                       : run_moments_bf16<9>(*plan, row_ptr, H_on, H_bond, mu, w, lay, stream);
    if (plan->dtype == BOP_F64)
        return no == 5 ? run_moments<double, 5>(*plan, row_ptr, H_on, H_bond, mu, w, lay, stream)
                       : run_moments<double, 9>(*plan, row_ptr, H_on, H_bond, mu, w, lay, stream);
    return no == 5 ? run_moments<float, 5>(*plan, row_ptr, H_on, H_bond, mu, w, lay, stream)
                   : run_moments<float, 9>(*plan, row_ptr, H_on, H_bond, mu, w, lay, stream);
}

extern "C" int bop_lanczos(const bop_plan *plan, const int *row_ptr, const double *H_on, const void *H_bond,
                           double *a, double *b, int *flags, void *ws, size_t ws_bytes, hipStream_t stream)
{
    BOP_REQUIRE(plan, BOP_E_ARG, "bop_lanczos: plan is NULL");
    BOP_REQUIRE(ws && ws_bytes >= plan->ws_bytes, BOP_E_CAPACITY,
                "bop_lanczos: workspace of %zu bytes needed, %zu given", plan->ws_bytes, ws_bytes);
    const int n = plan->n_atoms, no = plan->n_orb;
    if (n == 0) return BOP_OK;
    BOP_REQUIRE(row_ptr && H_on && H_bond && b && flags && (a || plan->n_max == 0), BOP_E_ARG,
                "bop_lanczos: NULL array");
    Layout lay = make_layout(*plan, map_workgroups(n, plan->n_tiles));
    char *w = (char *)ws;
    // BF16 or FP16 vectors, d band, at most 16 neighbours per row: the fused
    // MFMA pass on packed rows; otherwise BF16 takes the two-pass form on
    // padded rows and FP16 the FP32 pass with FP16 storage
    if ((plan->dtype == BOP_BF16 || plan->dtype == BOP_F16) && no == 5 && plan->deg_max <= 16)
        return plan->dtype == BOP_BF16 ? run_lanczos16<false>(*plan, row_ptr, H_on, H_bond, a, b, flags, w, lay, stream)
                                       : run_lanczos16<true>(*plan, row_ptr, H_on, H_bond, a, b, flags, w, lay, stream);
    if (plan->dtype == BOP_BF16)
        return no == 5 ? run_lanczos_bf16<5>(*plan, row_ptr, H_on, H_bond, a, b, flags, w, lay, stream)
                       : run_lanczos_bf16<9>(*plan, row_ptr, H_on, H_bond, a, b, flags, w, lay, stream);
    if (plan->dtype == BOP_F64)
        return no == 5 ? run_lanczos<double, 5>(*plan, row_ptr, H_on, H_bond, a, b, flags, w, lay, stream)
                       : run_lanczos<double, 9>(*plan, row_ptr, H_on, H_bond, a, b, flags, w, lay, stream);
    if (plan->dtype == BOP_F16)
        return no == 5 ? run_lanczos<float, 5, _Float16>(*plan, row_ptr, H_on, H_bond, a, b, flags, w, lay, stream)
                       : run_lanczos<float, 9, _Float16>(*plan, row_ptr, H_on, H_bond, a, b, flags, w, lay, stream);
    return no == 5 ? run_lanczos<float, 5>(*plan, row_ptr, H_on, H_bond, a, b, flags, w, lay, stream)
                   : run_lanczos<float, 9>(*plan, row_ptr, H_on, H_bond, a, b, flags, w, lay, stream);
}
