// Orbital moments mu_ia^(n) = <i a|H^n|i a> (App. B.3 of arXiv:1803.07491,
// Eq. momDOS), computed from interference paths built iteratively,
// X^k = H X^(k-1) (Eq. xi_rec), and merged at the middle of each path
// (Eqs. xi_invert, xi_merge):
//     mu_2k = <X^k, X^k>,  mu_2k-1 = <X^(k-1), X^k>,  mu_2K+1 = <X^K, H X^K>.
//
// GPU design (not the paper's CPU scheme):
//  * A tile is a group of B spatially adjacent atoms; the B * n_orb unit start
//    vectors are the columns of X, one column per lane of a 64-wide wavefront.
//  * A persistent workgroup takes tiles from a device queue.  For each tile it
//    first finds the k-hop support with a deterministic breadth-first search:
//    every frontier (row, slot) claims its neighbour with an atomic minimum on
//    a per-workgroup global->local map, and the owners are compacted in
//    (row, slot) order, so local rows come out in layer order and the result is
//    independent of scheduling.  Each local row keeps its neighbour slots
//    sorted by the neighbour's layer: at step k the neighbours whose X^(k-1) is
//    non-zero form a prefix of that list.
//  * Step k runs over the rows of the k-hop support; a wavefront owns a row and
//    all 64 columns.  The row's H blocks are wave-uniform and come in through
//    scalar loads; the neighbour rows of X^(k-1) are coalesced vector loads.
//    The moment dot products are fused into the step and reduced across the
//    workgroup's wavefronts in a fixed order (deterministic, FP64).
//  * X lives in the workgroup's slice of the workspace (HBM, L2-resident per
//    tile step), ping-ponged between two buffers.
#include "bop_internal.h"

namespace bop {
namespace {

constexpr int UNSEEN = 0x7fffffff;
constexpr int CLAIM = 1 << 30;
constexpr int MAX_NMAX = 40;
constexpr int MAXK = MAX_NMAX / 2;
constexpr int HDR = 256;            // header: [0] queue, [1] error, [2] max rows, [3] max degree
constexpr int PLAN_WG = 64, PLAN_T = 256;

struct WgLayout {
    size_t g2l, sup, rinfo, lnb, x0, x1, bytes;
};

__host__ __device__ inline WgLayout wg_layout(int n_atoms, int rows_cap, int deg_max, int no, int tsize)
{
    WgLayout L;
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += (b + 255) / 256 * 256; return r; };
    L.g2l = take(4ull * n_atoms);
    L.sup = take(4ull * rows_cap);
    L.rinfo = take(4ull * rows_cap);
    L.lnb = take(4ull * rows_cap * deg_max);
    L.x0 = take((size_t)tsize * rows_cap * no * 64);
    L.x1 = take((size_t)tsize * rows_cap * no * 64);
    L.bytes = o;
    return L;
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
template <int WGT>
__device__ int bfs_tile(int tile, int B, int n_atoms, int K, const int *__restrict__ order,
                        const int *__restrict__ row_ptr, const int *__restrict__ nbr_j, int deg_max,
                        int *g2l, int *sup, int rows_cap, int *s_size, int *s_wave, int *s_flag)
{
    const int tid = threadIdx.x;
    const int first = tile * B;
    const int Bt = min(B, n_atoms - first);
    if (tid < Bt && tid < rows_cap) {
        int g = order ? order[first + tid] : first + tid;
        sup[tid] = g;
        atomic_store_agent(&g2l[g], tid);
    }
    if (tid == 0) { s_size[0] = Bt; s_flag[0] = 0; }
    __syncthreads();
    if (Bt > rows_cap) {
        for (int t = tid; t < rows_cap; t += WGT) atomic_store_agent(&g2l[sup[t]], UNSEEN);
        __syncthreads();
        return -1;
    }
    for (int k = 1; k <= K; ++k) {
        const int begin = (k >= 2) ? s_size[k - 2] : 0, end = s_size[k - 1];
        const long nent = (long)(end - begin) * deg_max;
        for (long e = tid; e < nent; e += WGT) {
            int t = begin + (int)(e / deg_max), s = (int)(e % deg_max);
            int g = sup[t];
            int p0 = row_ptr[g], deg = row_ptr[g + 1] - p0;
            if (s < deg) atomicMin(&g2l[nbr_j[p0 + s]], CLAIM + (int)e);
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
                    own = atomic_load_agent(&g2l[j]) == CLAIM + (int)e;
                }
            }
            int tot;
            int pos = wg_scan01<WGT>(own, s_wave, tot);
            if (own) {
                int idx = base + pos;
                if (idx < rows_cap) { sup[idx] = j; atomic_store_agent(&g2l[j], idx); }
                else s_flag[0] = 1;
            }
            base += tot;
        }
        __syncthreads();
        if (s_flag[0]) {
            // restore the map: every claimed atom neighbours this frontier
            for (int t = tid; t < min(base, rows_cap); t += WGT) atomic_store_agent(&g2l[sup[t]], UNSEEN);
            for (long e = tid; e < nent; e += WGT) {
                int t = begin + (int)(e / deg_max), s = (int)(e % deg_max);
                int g = sup[t];
                int p0 = row_ptr[g], deg = row_ptr[g + 1] - p0;
                if (s < deg) atomic_store_agent(&g2l[nbr_j[p0 + s]], UNSEEN);
            }
            __syncthreads();
            return -1;
        }
        if (tid == 0) s_size[k] = base;
        __syncthreads();
    }
    return s_size[K];
}

template <int WGT>
__device__ inline void reset_map(int *g2l, const int *sup, int rows)
{
    for (int t = threadIdx.x; t < rows; t += WGT) atomic_store_agent(&g2l[sup[t]], UNSEEN);
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
       int *hdr, char *scratch, size_t per_wg)
{
    __shared__ int s_size[MAXK + 2], s_wave[PLAN_T / 64], s_flag[1], s_tile[1];
    char *mine = scratch + per_wg * blockIdx.x;
    int *g2l = (int *)mine;
    int *sup = (int *)(mine + align_up(4ull * n_atoms, 256));
    for (;;) {
        int tile = next_tile(&hdr[0], s_tile);
        if (tile >= n_tiles) break;
        int rows = bfs_tile<PLAN_T>(tile, B, n_atoms, K, order, row_ptr, nbr_j, deg_max, g2l, sup,
                                    n_atoms, s_size, s_wave, s_flag);
        if (threadIdx.x == 0) atomicMax(&hdr[2], rows);
        reset_map<PLAN_T>(g2l, sup, rows);
    }
}

__global__ void k_max_degree(int n, const int *__restrict__ row_ptr, int *hdr)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int d = (i < n) ? row_ptr[i + 1] - row_ptr[i] : 0;
    for (int o = 32; o > 0; o >>= 1) d = max(d, __shfl_xor(d, o));
    if ((threadIdx.x & 63) == 0) atomicMax(&hdr[3], d);
}

__global__ void k_init(int *hdr, int *maps, long n_map)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 4) hdr[i] = 0;
    if (i < n_map) maps[i] = UNSEEN;
}

__global__ void k_init_strided(int *hdr, char *base, size_t stride, int n_wg, int n_atoms)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2) hdr[i] = 0;
    long total = (long)n_wg * n_atoms;
    if (i < total) {
        long w = i / n_atoms, a = i % n_atoms;
        ((int *)(base + stride * w))[a] = UNSEEN;
    }
}

// ---------------------------------------------------------------------------
// moments
// ---------------------------------------------------------------------------
template <typename T> __device__ inline T from_f64(double v) { return (T)v; }

template <typename T, int NO, int WGT>
__global__ void __launch_bounds__(WGT)
k_moments(int n_atoms, int n_max, int B, int n_tiles, const int *__restrict__ order,
          const int *__restrict__ row_ptr, const int *__restrict__ nbr_j,
          const double *__restrict__ H_on, const T *__restrict__ H,
          double *__restrict__ mu, int *hdr, char *ws, size_t per_wg, WgLayout lay,
          int rows_cap, int deg_max)
{
    constexpr int NW = WGT / 64;
    __shared__ int s_size[MAXK + 2], s_wave[NW], s_flag[1], s_tile[1];
    __shared__ double s_red[2][NW][64];
    const int K = n_max / 2;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    char *mine = ws + per_wg * blockIdx.x;
    int *g2l = (int *)(mine + lay.g2l);
    int *sup = (int *)(mine + lay.sup);
    int *rinfo = (int *)(mine + lay.rinfo);
    int *lnb = (int *)(mine + lay.lnb);
    T *X0 = (T *)(mine + lay.x0);
    T *X1 = (T *)(mine + lay.x1);
    const int stride_row = NO * 64;
    const int n1m = n_max + 1;

    for (;;) {
        const int tile = next_tile(&hdr[0], s_tile);
        if (tile >= n_tiles) break;
        const int first = tile * B;
        const int Bt = min(B, n_atoms - first);
        const int rows = bfs_tile<WGT>(tile, B, n_atoms, K, order, row_ptr, nbr_j, deg_max, g2l, sup,
                                       rows_cap, s_size, s_wave, s_flag);
        if (rows < 0) {                      // support larger than planned
            if (threadIdx.x == 0) atomicOr(&hdr[1], 1);
            for (int c = threadIdx.x; c < Bt * NO * n1m; c += WGT) {
                int b = c / (NO * n1m), rest = c % (NO * n1m);
                int g = order ? order[first + b] : first + b;
                mu[(long)g * NO * n1m + rest] = __builtin_nan("");
            }
            __syncthreads();
            continue;
        }
        // --- per-row layer and layer-sorted neighbour slots -----------------
        for (int l = threadIdx.x; l < rows; l += WGT) {
            int g = sup[l];
            int L = 0;
            while (l >= s_size[L]) ++L;
            const int lo = (L >= 1) ? s_size[L - 1] : 0;   // rows below layer L start here
            const int endL = s_size[L];
            const int endL1 = (L + 1 <= K) ? s_size[L + 1] : s_size[K];
            int p0 = row_ptr[g], deg = row_ptr[g + 1] - p0;
            int *dst = lnb + (long)l * deg_max;
            int c = 0, n1 = 0, n2 = 0;
            for (int pass = 0; pass < 3; ++pass) {
                for (int s = 0; s < deg; ++s) {
                    int lj = atomic_load_agent(&g2l[nbr_j[p0 + s]]);
                    int cls = (lj < lo) ? 0 : (lj < endL ? 1 : (lj < endL1 ? 2 : 3));
                    if (cls == pass) dst[c++] = (lj << 8) | s;
                }
                if (pass == 0) n1 = c;
                if (pass == 1) n2 = c;
            }
            rinfo[l] = L | (n1 << 8) | (n2 << 16) | (c << 24);
        }
        // --- X^0 = unit columns; mu_0 = 1 -----------------------------------
        for (int l = w; l < Bt; l += NW)
#pragma unroll
            for (int a = 0; a < NO; ++a)
                X0[(long)l * stride_row + a * 64 + lane] = (lane == l * NO + a) ? T(1) : T(0);
        if (threadIdx.x < Bt * NO) {
            int b = threadIdx.x / NO, a = threadIdx.x % NO;
            mu[((long)sup[b] * NO + a) * n1m] = 1.0;
        }
        __syncthreads();

        T *Xp = X0, *Xc = X1;
        const int steps = K + (n_max & 1);
        for (int k = 1; k <= steps; ++k) {
            const bool last = k > K;
            const int nrow = last ? s_size[K] : s_size[k];
            double so = 0.0, se = 0.0;
            for (int l = w; l < nrow; l += NW) {
                const int g = __builtin_amdgcn_readfirstlane(sup[l]);
                const int info = __builtin_amdgcn_readfirstlane(rinfo[l]);
                const int L = info & 255, n1 = (info >> 8) & 255, n2 = (info >> 16) & 255,
                          n3 = (info >> 24) & 255;
                const bool has_prev = last || L <= k - 1;
                const int nval = last ? n3 : (k - 1 >= L + 1 ? n3 : (k - 1 == L ? n2 : n1));
                const int p0 = row_ptr[g];
                const T *xrow = Xp + (long)l * stride_row + lane;
                T acc[NO], xs[NO];
#pragma unroll
                for (int a = 0; a < NO; ++a) {
                    xs[a] = has_prev ? xrow[a * 64] : T(0);
                    acc[a] = from_f64<T>(H_on[(long)g * NO + a]) * xs[a];
                }
                const int slots = (lane < nval) ? lnb[(long)l * deg_max + lane] : 0;
                for (int s = 0; s < nval; ++s) {
                    const int pk = __builtin_amdgcn_readlane(slots, s);
                    const T *xn = Xp + (long)(pk >> 8) * stride_row + lane;
                    const T *h = H + (long)(p0 + (pk & 255)) * (NO * NO);
                    T x[NO];
#pragma unroll
                    for (int b = 0; b < NO; ++b) x[b] = xn[b * 64];
#pragma unroll
                    for (int a = 0; a < NO; ++a)
#pragma unroll
                        for (int b = 0; b < NO; ++b) acc[a] = fma(h[a * NO + b], x[b], acc[a]);
                }
                if (!last) {
                    T *xo = Xc + (long)l * stride_row + lane;
#pragma unroll
                    for (int a = 0; a < NO; ++a) xo[a * 64] = acc[a];
                }
#pragma unroll
                for (int a = 0; a < NO; ++a) {
                    so = fma((double)xs[a], (double)acc[a], so);
                    se = fma((double)acc[a], (double)acc[a], se);
                }
            }
            s_red[0][w][lane] = so;
            s_red[1][w][lane] = se;
            __syncthreads();
            if (threadIdx.x < Bt * NO) {
                double to = 0.0, te = 0.0;
#pragma unroll
                for (int q = 0; q < NW; ++q) { to += s_red[0][q][threadIdx.x]; te += s_red[1][q][threadIdx.x]; }
                int b = threadIdx.x / NO, a = threadIdx.x % NO;
                double *m = mu + ((long)sup[b] * NO + a) * n1m;
                if (last) m[2 * K + 1] = to;
                else { m[2 * k - 1] = to; m[2 * k] = te; }
            }
            __syncthreads();
            if (!last) { T *t = Xp; Xp = Xc; Xc = t; }
        }
        reset_map<WGT>(g2l, sup, rows);
    }
}

template <typename T, int NO>
hipError_t launch_moments(int wgt, dim3 grid, hipStream_t st, int n_atoms, int n_max, int B, int n_tiles,
                          const int *order, const int *row_ptr, const int *nbr_j, const double *H_on,
                          const void *H, double *mu, int *hdr, char *ws, size_t per_wg, WgLayout lay,
                          int rows_cap, int deg_max)
{
#define BOP_LAUNCH_M(W)                                                                             \
    k_moments<T, NO, W><<<grid, W, 0, st>>>(n_atoms, n_max, B, n_tiles, order, row_ptr, nbr_j, H_on, \
                                            (const T *)H, mu, hdr, ws, per_wg, lay, rows_cap, deg_max)
    if (wgt == 256) BOP_LAUNCH_M(256);
    else if (wgt == 512) BOP_LAUNCH_M(512);
    else BOP_LAUNCH_M(1024);
#undef BOP_LAUNCH_M
    return hipGetLastError();
}

int default_tile_atoms(int no) { return 64 / no; }

}  // namespace
}  // namespace bop

using namespace bop;

extern "C" size_t bop_moments_plan_scratch_size(int n_atoms)
{
    if (n_atoms < 0) return 0;
    size_t per = align_up(4ull * n_atoms, 256) * 2;
    return HDR + PLAN_WG * per;
}

extern "C" int bop_moments_plan(int n_atoms, int n_orb, int n_max, int dtype, const int *row_ptr,
                                const int *nbr_j, const int *order, const bop_tuning *tuning,
                                void *scratch, size_t scratch_bytes, bop_plan *plan,
                                hipStream_t stream)
{
    BOP_REQUIRE(plan && n_atoms >= 0, BOP_E_ARG, "bop_moments_plan: bad arguments");
    BOP_REQUIRE(n_orb == 5 || n_orb == 9, BOP_E_UNSUPPORTED, "bop_moments_plan: n_orb must be 5 or 9");
    BOP_REQUIRE(n_max >= 0 && n_max <= MAX_NMAX, BOP_E_UNSUPPORTED, "bop_moments_plan: n_max must be 0..%d", MAX_NMAX);
    BOP_REQUIRE(dtype == BOP_F64 || dtype == BOP_F32, BOP_E_UNSUPPORTED,
                "bop_moments_plan: dtype %d not supported by the vector kernel", dtype);
    BOP_REQUIRE(n_atoms == 0 || (row_ptr && nbr_j), BOP_E_ARG, "bop_moments_plan: neighbour arrays NULL");
    size_t need = bop_moments_plan_scratch_size(n_atoms);
    BOP_REQUIRE(scratch && scratch_bytes >= need, BOP_E_CAPACITY,
                "bop_moments_plan: scratch of %zu bytes needed", need);
    int B = (tuning && tuning->tile_atoms > 0) ? tuning->tile_atoms : default_tile_atoms(n_orb);
    BOP_REQUIRE(B * n_orb <= 64, BOP_E_UNSUPPORTED, "bop_moments_plan: tile_atoms * n_orb must be <= 64");
    int wgt = (tuning && tuning->block_threads) ? tuning->block_threads : 512;
    BOP_REQUIRE(wgt == 256 || wgt == 512 || wgt == 1024, BOP_E_UNSUPPORTED,
                "bop_moments_plan: block_threads must be 256, 512 or 1024");
    int nwg = (tuning && tuning->n_blocks > 0) ? tuning->n_blocks : 2 * device_cus();
    int n_tiles = (n_atoms + B - 1) / B;
    if (nwg > n_tiles) nwg = n_tiles > 0 ? n_tiles : 1;

    int *hdr = (int *)scratch;
    char *base = (char *)scratch + HDR;
    size_t per = align_up(4ull * n_atoms, 256) * 2;
    long nmap = (long)PLAN_WG * (long)(per / 4);
    k_init<<<(unsigned)((nmap + 255) / 256 > 0 ? (nmap + 255) / 256 : 1), 256, 0, stream>>>(hdr, (int *)base, nmap);
    BOP_LAUNCHED();
    int hv[4] = { 0, 0, 0, 0 };
    if (n_atoms > 0) {
        k_max_degree<<<(n_atoms + 255) / 256, 256, 0, stream>>>(n_atoms, row_ptr, hdr);
        BOP_LAUNCHED();
        BOP_HIP(hipMemcpyAsync(hv, hdr, sizeof hv, hipMemcpyDeviceToHost, stream));
        BOP_HIP(hipStreamSynchronize(stream));
        BOP_REQUIRE(hv[3] <= 64, BOP_E_UNSUPPORTED, "bop_moments_plan: %d neighbours in a row (at most 64)", hv[3]);
        int dmax = hv[3] > 0 ? hv[3] : 1;
        int pwg = n_tiles < PLAN_WG ? (n_tiles > 0 ? n_tiles : 1) : PLAN_WG;
        k_plan<<<pwg, PLAN_T, 0, stream>>>(n_atoms, B, n_tiles, n_max / 2, order, row_ptr, nbr_j, dmax,
                                           hdr, base, per);
        BOP_LAUNCHED();
        BOP_HIP(hipMemcpyAsync(hv, hdr, sizeof hv, hipMemcpyDeviceToHost, stream));
        BOP_HIP(hipStreamSynchronize(stream));
    }
    plan->n_atoms = n_atoms;
    plan->n_orb = n_orb;
    plan->n_max = n_max;
    plan->dtype = dtype;
    plan->tile_atoms = B;
    plan->n_tiles = n_tiles;
    plan->block_threads = wgt;
    plan->n_blocks = nwg;
    plan->deg_max = hv[3] > 0 ? hv[3] : 1;
    plan->rows_cap = hv[2] > 0 ? hv[2] : 1;
    BOP_REQUIRE(plan->rows_cap < (1 << 23), BOP_E_UNSUPPORTED, "bop_moments_plan: tile support too large");
    WgLayout lay = wg_layout(n_atoms, plan->rows_cap, plan->deg_max, n_orb, dtype == BOP_F64 ? 8 : 4);
    plan->ws_bytes = HDR + (size_t)nwg * lay.bytes;
    return BOP_OK;
}

extern "C" int bop_moments(const bop_plan *plan, const int *row_ptr, const int *nbr_j,
                           const int *order, const double *H_on, const void *H_bond, double *mu,
                           void *ws, size_t ws_bytes, hipStream_t stream)
{
    BOP_REQUIRE(plan, BOP_E_ARG, "bop_moments: plan is NULL");
    const int n = plan->n_atoms, no = plan->n_orb;
    BOP_REQUIRE(ws && ws_bytes >= plan->ws_bytes, BOP_E_CAPACITY,
                "bop_moments: workspace of %zu bytes needed, %zu given", plan->ws_bytes, ws_bytes);
    if (n == 0) return BOP_OK;
    BOP_REQUIRE(row_ptr && nbr_j && H_on && H_bond && mu, BOP_E_ARG, "bop_moments: NULL array");
    const int tsize = plan->dtype == BOP_F64 ? 8 : 4;
    WgLayout lay = wg_layout(n, plan->rows_cap, plan->deg_max, no, tsize);
    int *hdr = (int *)ws;
    char *base = (char *)ws + HDR;
    long tot = (long)plan->n_blocks * n;
    k_init_strided<<<(unsigned)((tot + 255) / 256), 256, 0, stream>>>(hdr, base + lay.g2l, lay.bytes,
                                                                       plan->n_blocks, n);
    BOP_LAUNCHED();
    dim3 grid(plan->n_blocks);
    hipError_t e;
    if (plan->dtype == BOP_F64) {
        if (no == 5) e = launch_moments<double, 5>(plan->block_threads, grid, stream, n, plan->n_max, plan->tile_atoms, plan->n_tiles, order, row_ptr, nbr_j, H_on, H_bond, mu, hdr, base, lay.bytes, lay, plan->rows_cap, plan->deg_max);
        else e = launch_moments<double, 9>(plan->block_threads, grid, stream, n, plan->n_max, plan->tile_atoms, plan->n_tiles, order, row_ptr, nbr_j, H_on, H_bond, mu, hdr, base, lay.bytes, lay, plan->rows_cap, plan->deg_max);
    } else {
        if (no == 5) e = launch_moments<float, 5>(plan->block_threads, grid, stream, n, plan->n_max, plan->tile_atoms, plan->n_tiles, order, row_ptr, nbr_j, H_on, H_bond, mu, hdr, base, lay.bytes, lay, plan->rows_cap, plan->deg_max);
        else e = launch_moments<float, 9>(plan->block_threads, grid, stream, n, plan->n_max, plan->tile_atoms, plan->n_tiles, order, row_ptr, nbr_j, H_on, H_bond, mu, hdr, base, lay.bytes, lay, plan->rows_cap, plan->deg_max);
    }
    BOP_REQUIRE(e == hipSuccess, BOP_E_HIP, "bop_moments: launch failed: %s", hipGetErrorString(e));
    return BOP_OK;
}
