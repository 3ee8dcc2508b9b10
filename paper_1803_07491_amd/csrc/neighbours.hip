// Periodic neighbour list on the GPU (Sec. II "Initialisation" of
// arXiv:1803.07491: pairs within the cutoff found through cell lists, the
// ghost cells of the paper expressed as explicit integer image shifts S).
//
// Atoms are binned into a grid of cells at least r_cut wide (in fractional
// coordinates along each reciprocal direction), cells numbered in 2x2x2
// blocks.  The atom order emitted for moment tiles follows a Hilbert curve
// over a grid three times finer (index order inside a grid cell): consecutive
// atoms then form compact groups, whose union of k-hop neighbourhoods is ~5%
// smaller than for groups taken in cell-list order.  Each atom then scans the 27 neighbouring
// cells; the image shift of a candidate follows from the cell wrap and the
// atoms' integer offsets.  If some axis has fewer than three cells, every atom
// scans all atoms and all image shifts that can reach the cutoff.
//
// The pair vector and the criterion are evaluated in one fixed operation
// order in FP64 with contraction disabled for this file, so the list is
// bit-exact; rows are sorted by (j, s1, s2, s3).
#include "bop_internal.h"

#include <cmath>

namespace bop {
namespace {

struct Geom {
    double A[9];      // rows a1, a2, a3
    double Ai[9];     // inverse: f = r . Ai
    double gn[3];     // |column k of Ai| = 1 / plane spacing
    int nc[3];        // cells per axis
    int nb[3];        // 2x2x2 blocks per axis
    int nt[3];        // tile-order grid per axis (Hilbert curve of tb bits per axis)
    int tb;
    double rc, rc2;
    int all_pairs;    // 1: brute-force over atoms and shifts
};

__host__ __device__ inline int bin_of_cell(const Geom &g, int c0, int c1, int c2)
{
    int blk = ((c0 >> 1) * g.nb[1] + (c1 >> 1)) * g.nb[2] + (c2 >> 1);
    return blk * 8 + ((c0 & 1) << 2) + ((c1 & 1) << 1) + (c2 & 1);
}

// d = (r_j - r_i) + ((s1 a1 + s2 a2) + s3 a3);  accepted when 0 < |d|^2 < rc^2
__device__ inline bool pair_vec(const Geom &g, const double *__restrict__ pos, int i, int j,
                                int s1, int s2, int s3, double d[3])
{
    for (int k = 0; k < 3; ++k) {
        double sv = ((double)s1 * g.A[k] + (double)s2 * g.A[3 + k]) + (double)s3 * g.A[6 + k];
        d[k] = (pos[3 * j + k] - pos[3 * i + k]) + sv;
    }
    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    return r2 > 0.0 && r2 < g.rc2;
}

__global__ void k_fill_int(int *p, long n, int v)
{
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// 3-D Hilbert index of (x0, x1, x2), b bits each (Skilling's transpose
// method: undo the excess work per bit plane, Gray-encode, interleave).
__device__ inline unsigned hilbert3(unsigned x0, unsigned x1, unsigned x2, int b)
{
    unsigned X[3] = {x0, x1, x2};
    const unsigned M = 1u << (b - 1);
    for (unsigned Q = M; Q > 1; Q >>= 1) {
        const unsigned P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) X[0] ^= P;
            else {
                const unsigned t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    unsigned t = 0;
    for (unsigned Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    unsigned code = 0;
    for (int bit = b - 1; bit >= 0; --bit)
        for (int i = 0; i < 3; ++i) code = (code << 1) | ((X[i] >> bit) & 1u);
    return code;
}

// tile-order key: Hilbert index of the atom's cell in the fine grid
__global__ void k_tile_key(Geom g, int n, const double *__restrict__ f, const int *__restrict__ u,
                           int *__restrict__ key, int *__restrict__ key_count)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned c[3];
    for (int k = 0; k < 3; ++k) {
        const double w = f[3 * i + k] - (double)u[3 * i + k];
        int ck = (int)(w * g.nt[k]);
        ck = ck < 0 ? 0 : (ck >= g.nt[k] ? g.nt[k] - 1 : ck);
        c[k] = (unsigned)ck;
    }
    const int h = (int)hilbert3(c[0], c[1], c[2], g.tb);
    key[i] = h;
    atomicAdd(&key_count[h], 1);
}

__global__ void k_bin_atoms(Geom g, int n, const double *__restrict__ pos, double *__restrict__ f,
                            int *__restrict__ u, int *__restrict__ cellc, int *__restrict__ bin,
                            int *__restrict__ bin_count)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c[3];
    for (int k = 0; k < 3; ++k) {
        double fk = pos[3 * i] * g.Ai[k] + pos[3 * i + 1] * g.Ai[3 + k] + pos[3 * i + 2] * g.Ai[6 + k];
        double uk = floor(fk);
        double w = fk - uk;
        int ck = (int)(w * g.nc[k]);
        ck = ck < 0 ? 0 : (ck >= g.nc[k] ? g.nc[k] - 1 : ck);
        f[3 * i + k] = fk;
        u[3 * i + k] = (int)uk;
        c[k] = ck;
    }
    cellc[i] = (c[0] << 20) | (c[1] << 10) | c[2];
    int b = bin_of_cell(g, c[0], c[1], c[2]);
    bin[i] = b;
    atomicAdd(&bin_count[b], 1);
}

__global__ void k_fill_bins(int n, const int *__restrict__ bin, const int *__restrict__ bin_start,
                            int *__restrict__ cursor, int *__restrict__ bin_list)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = bin[i];
    int s = atomicAdd(&cursor[b], 1);
    bin_list[bin_start[b] + s] = i;
}

// sort each bin's atoms by index (deterministic cell lists and atom order)
__global__ void k_sort_bins(long nbins, const int *__restrict__ bin_start, int *__restrict__ bin_list)
{
    long b = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    int lo = bin_start[b], hi = bin_start[b + 1];
    for (int t = lo + 1; t < hi; ++t) {
        int v = bin_list[t], s = t - 1;
        while (s >= lo && bin_list[s] > v) { bin_list[s + 1] = bin_list[s]; --s; }
        bin_list[s + 1] = v;
    }
}

// Candidate enumeration shared by the count and fill passes.  For each
// accepted (j, S) calls emit(j, s1, s2, s3, d).
template <typename Emit>
__device__ inline void scan_atom(const Geom &g, int n, int i, const double *__restrict__ pos,
                                 const double *__restrict__ f, const int *__restrict__ u,
                                 const int *__restrict__ cellc, const int *__restrict__ bin_start,
                                 const int *__restrict__ bin_list, Emit emit)
{
    if (g.all_pairs) {
        for (int j = 0; j < n; ++j) {
            int lo[3], hi[3];
            for (int k = 0; k < 3; ++k) {
                double df = f[3 * j + k] - f[3 * i + k];
                lo[k] = (int)ceil(-g.rc * g.gn[k] - df) - 1;
                hi[k] = (int)floor(g.rc * g.gn[k] - df) + 1;
            }
            for (int s1 = lo[0]; s1 <= hi[0]; ++s1)
                for (int s2 = lo[1]; s2 <= hi[1]; ++s2)
                    for (int s3 = lo[2]; s3 <= hi[2]; ++s3) {
                        double d[3];
                        if (pair_vec(g, pos, i, j, s1, s2, s3, d)) emit(j, s1, s2, s3, d);
                    }
        }
        return;
    }
    int cc = cellc[i];
    int ci[3] = { cc >> 20, (cc >> 10) & 1023, cc & 1023 };
    int ui[3] = { u[3 * i], u[3 * i + 1], u[3 * i + 2] };
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                int c[3] = { ci[0] + dx, ci[1] + dy, ci[2] + dz }, w[3];
                for (int k = 0; k < 3; ++k) {
                    w[k] = 0;
                    if (c[k] < 0) { c[k] += g.nc[k]; w[k] = -1; }
                    else if (c[k] >= g.nc[k]) { c[k] -= g.nc[k]; w[k] = 1; }
                }
                int b = bin_of_cell(g, c[0], c[1], c[2]);
                for (int t = bin_start[b]; t < bin_start[b + 1]; ++t) {
                    int j = bin_list[t];
                    // the candidate sits at fractional f_j - u_j + w relative to
                    // f_i - u_i, so S = w + u_i - u_j
                    int s1 = w[0] + ui[0] - u[3 * j];
                    int s2 = w[1] + ui[1] - u[3 * j + 1];
                    int s3 = w[2] + ui[2] - u[3 * j + 2];
                    double d[3];
                    if (pair_vec(g, pos, i, j, s1, s2, s3, d)) emit(j, s1, s2, s3, d);
                }
            }
}

__global__ void k_count(Geom g, int n, const double *__restrict__ pos, const double *__restrict__ f,
                        const int *__restrict__ u, const int *__restrict__ cellc,
                        const int *__restrict__ bin_start, const int *__restrict__ bin_list,
                        int *__restrict__ cnt)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    scan_atom(g, n, i, pos, f, u, cellc, bin_start, bin_list,
              [&](int, int, int, int, const double *) { ++c; });
    cnt[i] = c;
}

__device__ inline bool key_less(int ja, int a1, int a2, int a3, int jb, int b1, int b2, int b3)
{
    if (ja != jb) return ja < jb;
    if (a1 != b1) return a1 < b1;
    if (a2 != b2) return a2 < b2;
    return a3 < b3;
}

__global__ void k_fill(Geom g, int n, const double *__restrict__ pos, const double *__restrict__ f,
                       const int *__restrict__ u, const int *__restrict__ cellc,
                       const int *__restrict__ bin_start, const int *__restrict__ bin_list,
                       const int *__restrict__ row_ptr, int *__restrict__ nbr_j,
                       int *__restrict__ nbr_shift, double *__restrict__ nbr_d)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long base = row_ptr[i];
    int c = 0;
    // insertion into the row in sorted position as candidates arrive
    scan_atom(g, n, i, pos, f, u, cellc, bin_start, bin_list,
              [&](int j, int s1, int s2, int s3, const double *d) {
                  long t = base + c - 1;
                  while (t >= base && key_less(j, s1, s2, s3, nbr_j[t], nbr_shift[3 * t],
                                               nbr_shift[3 * t + 1], nbr_shift[3 * t + 2])) {
                      nbr_j[t + 1] = nbr_j[t];
                      nbr_shift[3 * t + 3] = nbr_shift[3 * t];
                      nbr_shift[3 * t + 4] = nbr_shift[3 * t + 1];
                      nbr_shift[3 * t + 5] = nbr_shift[3 * t + 2];
                      nbr_d[3 * t + 3] = nbr_d[3 * t];
                      nbr_d[3 * t + 4] = nbr_d[3 * t + 1];
                      nbr_d[3 * t + 5] = nbr_d[3 * t + 2];
                      --t;
                  }
                  ++t;
                  nbr_j[t] = j;
                  nbr_shift[3 * t] = s1; nbr_shift[3 * t + 1] = s2; nbr_shift[3 * t + 2] = s3;
                  nbr_d[3 * t] = d[0]; nbr_d[3 * t + 1] = d[1]; nbr_d[3 * t + 2] = d[2];
                  ++c;
              });
}

bool make_geom(const double *cell, double rc, Geom &g)
{
    for (int k = 0; k < 9; ++k) g.A[k] = cell[k];
    const double *A = cell;
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6])
               + A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
    double *B = g.Ai;
    B[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    B[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    g.rc = rc;
    g.rc2 = rc * rc;
    g.all_pairs = 0;
    for (int k = 0; k < 3; ++k) {
        g.gn[k] = std::sqrt(B[k] * B[k] + B[3 + k] * B[3 + k] + B[6 + k] * B[6 + k]);
        double m = std::floor(1.0 / (rc * g.gn[k] * (1.0 + 1e-9)));
        g.nc[k] = m < 1.0 ? 1 : (m > 1023.0 ? 1023 : (int)m);
        if (g.nc[k] < 3) g.all_pairs = 1;
        g.nb[k] = (g.nc[k] + 1) / 2;
        g.nt[k] = g.nc[k] * 3 > 256 ? 256 : g.nc[k] * 3;
    }
    int m = g.nt[0] > g.nt[1] ? g.nt[0] : g.nt[1];
    m = m > g.nt[2] ? m : g.nt[2];
    g.tb = 1;
    while ((1 << g.tb) < m) ++g.tb;
    return true;
}

struct NbrWs {
    double *f; int *u, *cellc, *bin, *bin_count, *bin_start, *cursor, *bin_list;
    int *key, *key_count, *key_start, *key_cursor;
    void *scan;
    size_t bytes;
};

NbrWs carve(void *base, int n, long nbins, long nkeys)
{
    NbrWs w{};
    char *p = (char *)base;
    auto take = [&](size_t b) { char *r = p; p += align_up(b, 256); return (void *)r; };
    w.f = (double *)take(sizeof(double) * 3 * (size_t)n);
    w.u = (int *)take(sizeof(int) * 3 * (size_t)n);
    w.cellc = (int *)take(sizeof(int) * (size_t)n);
    w.bin = (int *)take(sizeof(int) * (size_t)n);
    w.bin_count = (int *)take(sizeof(int) * (size_t)(nbins + 1));
    w.bin_start = (int *)take(sizeof(int) * (size_t)(nbins + 1));
    w.cursor = (int *)take(sizeof(int) * (size_t)(nbins + 1));
    w.bin_list = (int *)take(sizeof(int) * (size_t)n + 4);
    w.key = (int *)take(sizeof(int) * (size_t)n + 4);
    w.key_count = (int *)take(sizeof(int) * (size_t)(nkeys + 1));
    w.key_start = (int *)take(sizeof(int) * (size_t)(nkeys + 1));
    w.key_cursor = (int *)take(sizeof(int) * (size_t)(nkeys + 1));
    long sn = nbins > n ? nbins : n;
    sn = nkeys > sn ? nkeys : sn;
    w.scan = take(scan_scratch_bytes(sn + 1));
    w.bytes = (size_t)(p - (char *)base);
    return w;
}

}  // namespace
}  // namespace bop

using namespace bop;

extern "C" size_t bop_neighbours_workspace_size(int n_atoms, const double *cell, double r_cut)
{
    Geom g;
    if (n_atoms < 0 || !cell || !(r_cut > 0) || !make_geom(cell, r_cut, g)) return 0;
    long nbins = (long)g.nb[0] * g.nb[1] * g.nb[2] * 8;
    return carve(nullptr, n_atoms, nbins, 1L << (3 * g.tb)).bytes + 256;
}

extern "C" int bop_build_neighbours(int n, const double *pos, const double *cell, double r_cut,
                                    long capacity, int *row_ptr, int *nbr_j, int *nbr_shift,
                                    double *nbr_d, int *order, long *n_pairs,
                                    void *ws, size_t ws_bytes, hipStream_t stream)
{
    BOP_REQUIRE(n >= 0 && cell && n_pairs && row_ptr && capacity >= 0, BOP_E_ARG,
                "bop_build_neighbours: bad arguments");
    BOP_REQUIRE(n == 0 || pos, BOP_E_ARG, "bop_build_neighbours: pos is NULL");
    BOP_REQUIRE(r_cut > 0 && std::isfinite(r_cut), BOP_E_ARG, "bop_build_neighbours: r_cut must be > 0");
    Geom g;
    BOP_REQUIRE(make_geom(cell, r_cut, g), BOP_E_ARG, "bop_build_neighbours: singular cell");
    long nbins = (long)g.nb[0] * g.nb[1] * g.nb[2] * 8;
    const long nkeys = 1L << (3 * g.tb);
    NbrWs w = carve(ws, n, nbins, order ? nkeys : 0);
    BOP_REQUIRE(ws && ws_bytes >= w.bytes, BOP_E_CAPACITY,
                "bop_build_neighbours: workspace of %zu bytes needed, %zu given", w.bytes, ws_bytes);
    *n_pairs = 0;
    const int T = 256;
    auto blocks = [&](long m) { return (unsigned)((m + T - 1) / T > 0 ? (m + T - 1) / T : 1); };

    k_fill_int<<<blocks(nbins + 1), T, 0, stream>>>(w.bin_count, nbins + 1, 0);
    k_fill_int<<<blocks(nbins + 1), T, 0, stream>>>(w.cursor, nbins + 1, 0);
    BOP_LAUNCHED();
    if (n > 0) {
        k_bin_atoms<<<blocks(n), T, 0, stream>>>(g, n, pos, w.f, w.u, w.cellc, w.bin, w.bin_count);
        BOP_LAUNCHED();
    }
    int rc = exclusive_scan(w.bin_count, w.bin_start, nbins, w.scan, stream);
    if (rc) return rc;
    if (n > 0) {
        k_fill_bins<<<blocks(n), T, 0, stream>>>(n, w.bin, w.bin_start, w.cursor, w.bin_list);
        k_sort_bins<<<blocks(nbins), T, 0, stream>>>(nbins, w.bin_start, w.bin_list);
        BOP_LAUNCHED();
        if (order) {
            // tile order: counting sort of the atoms by Hilbert key, index order inside a key
            k_fill_int<<<blocks(nkeys + 1), T, 0, stream>>>(w.key_count, nkeys + 1, 0);
            k_fill_int<<<blocks(nkeys + 1), T, 0, stream>>>(w.key_cursor, nkeys + 1, 0);
            k_tile_key<<<blocks(n), T, 0, stream>>>(g, n, w.f, w.u, w.key, w.key_count);
            BOP_LAUNCHED();
            rc = exclusive_scan(w.key_count, w.key_start, nkeys, w.scan, stream);
            if (rc) return rc;
            k_fill_bins<<<blocks(n), T, 0, stream>>>(n, w.key, w.key_start, w.key_cursor, order);
            k_sort_bins<<<blocks(nkeys), T, 0, stream>>>(nkeys, w.key_start, order);
            BOP_LAUNCHED();
        }
        k_count<<<blocks(n), T, 0, stream>>>(g, n, pos, w.f, w.u, w.cellc, w.bin_start, w.bin_list, row_ptr);
        BOP_LAUNCHED();
    }
    rc = exclusive_scan(row_ptr, row_ptr, n, w.scan, stream);
    if (rc) return rc;
    int total = 0;
    BOP_HIP(hipMemcpyAsync(&total, row_ptr + n, sizeof(int), hipMemcpyDeviceToHost, stream));
    BOP_HIP(hipStreamSynchronize(stream));
    *n_pairs = total;
    BOP_REQUIRE(total >= 0, BOP_E_CAPACITY, "bop_build_neighbours: more than 2^31 pairs");
    if (total > capacity) {
        set_error("bop_build_neighbours: %d pairs, capacity %ld", total, capacity);
        return BOP_E_CAPACITY;
    }
    if (n > 0 && total > 0) {
        BOP_REQUIRE(nbr_j && nbr_shift && nbr_d, BOP_E_ARG, "bop_build_neighbours: output arrays are NULL");
        k_fill<<<blocks(n), T, 0, stream>>>(g, n, pos, w.f, w.u, w.cellc, w.bin_start, w.bin_list,
                                            row_ptr, nbr_j, nbr_shift, nbr_d);
        BOP_LAUNCHED();
    }
    return BOP_OK;
}
