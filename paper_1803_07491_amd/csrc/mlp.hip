// Learned warm start for the local-charge-neutrality cycle.  Not part of the
// paper; it generalises the paper's speed-up of starting the self-consistency
// from previously converged onsite levels (Sec. III "Speed-ups" (ii)) to a
// learned map from each atom's lowest moments to its converged onsite shift.
//
// Network (FP32): x (6) -> tanh(W1 x + b1) (64) -> tanh(W2 h1 + b2) (64)
//                 -> y = W3 h2 + b3 (1); loss = mean squared error.
// Parameters are one contiguous FP32 array:
//   W1[64][6] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3[1]   (4673 values)
//
// Kernels: features (per-atom moment traces, standardised), forward (row
// tiles of 16 per wave, the 64 x 64 layer on MFMA), and a training step made
// of a forward+backward pass over row tiles (both 64 x 64 products on MFMA),
// a per-block gradient reduction over rows (the W2 block on MFMA, the rest on
// the VALU), and an Adam update that sums the block partials in a fixed order
// (deterministic).
#include "bop_internal.h"

namespace bop {
namespace {

constexpr int NH = 64, NX = 6;
constexpr int OW1 = 0, OB1 = OW1 + NH * NX, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH, NPARAM = OB3 + 1;
static_assert(NPARAM == BOP_MLP_NPARAM, "parameter count");
constexpr int MT = 256;           // threads per block
constexpr int GRAD_BLOCKS = 64;   // row blocks of the gradient reduction (32: 74 us per 4,096-row step; 64: 57; 128: 73, Adam then summing more partials)

__device__ inline void load_params(const float *__restrict__ p, float *s)
{
    for (int e = threadIdx.x; e < NPARAM; e += blockDim.x) s[e] = p[e];
    __syncthreads();
}

// per-atom moment traces mu_i^(n) / n_orb, n = 1..6, standardised
__global__ void k_features(int n, int no, int n_max, const double *__restrict__ mu,
                           const float *__restrict__ mean, const float *__restrict__ stdv, float *__restrict__ x)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 1; k <= NX; ++k) {
        double s = 0.0;
        for (int a = 0; a < no; ++a) s += mu[((long)i * no + a) * (n_max + 1) + k];
        float v = (float)(s / no);
        if (mean) v = (v - mean[k - 1]) / stdv[k - 1];
        x[(long)i * NX + k - 1] = v;
    }
}

// Column statistics of the features x[n][NX]: block f computes feature f's
// mean and its standard deviation with the n - 1 normalisation (two passes,
// FP64 sums in a fixed order), the deviation floored at 1e-12.
__global__ void __launch_bounds__(MT)
k_feature_stats(int n, const float *__restrict__ x, float *__restrict__ mean, float *__restrict__ stdv)
{
    __shared__ double s_red[MT / 64];
    __shared__ double s_mean;
    const int f = blockIdx.x;
    double v = 0.0;
    for (long r = threadIdx.x; r < n; r += MT) v += (double)x[r * NX + f];
    v = block_combine(v, 0, s_red);
    if (threadIdx.x == 0) s_mean = v / (double)n;
    __syncthreads();
    const double m = s_mean;
    double q = 0.0;
    for (long r = threadIdx.x; r < n; r += MT) {
        const double d = (double)x[r * NX + f] - m;
        q = fma(d, d, q);
    }
    q = block_combine(q, 0, s_red);
    if (threadIdx.x == 0) {
        mean[f] = (float)m;
        const double sd = n > 1 ? sqrt(q / (double)(n - 1)) : 0.0;
        stdv[f] = (float)fmax(sd, 1e-12);
    }
}

__global__ void k_standardise(long n, const float *__restrict__ x, const float *__restrict__ mean,
                              const float *__restrict__ stdv, float *__restrict__ out)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * NX) return;
    const int f = (int)(e % NX);
    out[e] = (x[e] - mean[f]) / stdv[f];
}

// Gauge fix of predicted shifts: y -= mean(y), one block, FP64 sum in a fixed
// order (a shift common to all atoms moves E_F by the same amount and changes
// nothing else, so predictions are compared and used mean-free).
__global__ void __launch_bounds__(1024) k_remove_mean(int n, double *__restrict__ y)
{
    __shared__ double s_red[1024 / 64];
    __shared__ double s_mean;
    double v = 0.0;
    for (int r = threadIdx.x; r < n; r += blockDim.x) v += y[r];
    v = block_combine(v, 0, s_red);
    if (threadIdx.x == 0) s_mean = v / (double)n;
    __syncthreads();
    const double m = s_mean;
    for (int r = threadIdx.x; r < n; r += blockDim.x) y[r] -= m;
}

// partial gradients over one block of rows of every parameter but W2 (which
// k_mlp_grad_w2 sums on MFMA): thread (g, a) takes column a of the hidden
// layers and row group g (rows r0 + g, r0 + g + 4, ...), and sums W1[a][.],
// b1[a], b2[a], W3[a] (and b3 for a = 0) over them; the four row groups are
// then added in a fixed order.
__global__ void __launch_bounds__(MT)
k_mlp_grad(int B, const float *__restrict__ x, const float *__restrict__ H1, const float *__restrict__ H2,
           const float *__restrict__ GZ1, const float *__restrict__ GZ2, const float *__restrict__ GY,
           float *__restrict__ part)
{
    constexpr int NG = MT / NH;         // row groups
    constexpr int NV = NX + 4;          // W1 row, b1, b2, W3, b3
    __shared__ float s_p[NG][NV][NH];
    const int rows_per = (B + gridDim.x - 1) / gridDim.x;
    const int r0 = blockIdx.x * rows_per, r1 = min(B, r0 + rows_per);
    const int a = threadIdx.x % NH, g = threadIdx.x / NH;
    float v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.f;
    for (int r = r0 + g; r < r1; r += NG) {
        const float g1 = GZ1[(long)r * NH + a], g2 = GZ2[(long)r * NH + a], gy = GY[r];
#pragma unroll
        for (int c = 0; c < NX; ++c) v[c] = fmaf(g1, x[(long)r * NX + c], v[c]);
        v[NX] += g1;
        v[NX + 1] += g2;
        v[NX + 2] = fmaf(gy, H2[(long)r * NH + a], v[NX + 2]);
        v[NX + 3] += gy;
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) s_p[g][k][a] = v[k];
    __syncthreads();
    if (g == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            float t = s_p[0][k][a];
            for (int q = 1; q < NG; ++q) t += s_p[q][k][a];
            v[k] = t;
        }
        float *out = part + (size_t)blockIdx.x * NPARAM;
#pragma unroll
        for (int c = 0; c < NX; ++c) out[OW1 + a * NX + c] = v[c];
        out[OB1 + a] = v[NX];
        out[OB2 + a] = v[NX + 1];
        out[OW3 + a] = v[NX + 2];
        if (a == 0) out[OB3] = v[NX + 3];
    }
}

// sum of the block partials and Adam (lr, 0.9, 0.999, 1e-8): 64 parameters
// per workgroup, each summed by four threads over every fourth partial, the
// four sums then added in a fixed order
constexpr int AP = 64;                   // parameters per Adam workgroup

__global__ void __launch_bounds__(4 * AP)
k_mlp_adam(int nblk, int nloss, const float *__restrict__ part, const float *__restrict__ loss_part,
           float *__restrict__ params, float *__restrict__ m, float *__restrict__ v, int step, float lr,
           float *__restrict__ grad_out, float *__restrict__ loss)
{
    __shared__ float s_g[4][AP];
    const int pl = threadIdx.x % AP, grp = threadIdx.x / AP;
    const int p = blockIdx.x * AP + pl;
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
        float l = 0.f;
        for (int b = 0; b < nloss; ++b) l += loss_part[b];
        loss[0] = l;
    }
    float gp = 0.f;
    if (p < NPARAM)
        for (int b = grp; b < nblk; b += 4) gp += part[(size_t)b * NPARAM + p];
    s_g[grp][pl] = gp;
    __syncthreads();
    if (grp != 0 || p >= NPARAM) return;
    const float g = ((s_g[0][pl] + s_g[1][pl]) + s_g[2][pl]) + s_g[3][pl];
    if (grad_out) grad_out[p] = g;
    if (step <= 0) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float mm = b1 * m[p] + (1.f - b1) * g;
    float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    float mh = mm / (1.f - powf(b1, (float)step));
    float vh = vv / (1.f - powf(b2, (float)step));
    params[p] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_gather_rows(int B, const int *__restrict__ idx, const float *__restrict__ x,
                              const float *__restrict__ t, float *__restrict__ xb, float *__restrict__ tb)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= B) return;
    int s = idx[r];
#pragma unroll
    for (int c = 0; c < NX; ++c) xb[(long)r * NX + c] = x[(long)s * NX + c];
    tb[r] = t[s];
}

// ---------------------------------------------------------------------------
// MFMA forms.  The two 64 x 64 products of a row tile (H1 W2^T forward,
// GZ2 W2 backward) and the W2 gradient (sum over rows of GZ2^T H1) run on
// v_mfma_f32_16x16x4_f32 (FP32 operands, FP32 accumulation): one wave takes
// a tile of 16 rows; A[i][k] comes from lane i + 16 k, B[k][j] from lane
// j + 16 k, and the 4 results of lane l are D[4 (l / 16) + r][l % 16].  The
// 6 -> 64 and 64 -> 1 layers and the activations stay on the VALU.  W2 and
// the tiles sit in LDS with rows padded to 65 floats (conflict-free reads
// along either index).
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int RT = 16;          // rows per wave tile
constexpr int PS = NH + 1;      // padded LDS row

__device__ inline f4 mfma4(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

__device__ inline void lds_sync_wave()
{
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);     // this wave's LDS writes are done
    __builtin_amdgcn_wave_barrier();
}

// Forward (and with TRAIN the backward activations) of row tiles.  Without
// TRAIN: y[r] = network(x[r]).  With TRAIN: H1, H2, GZ1, GZ2, GY for the
// gradient pass and per-block partial sums of the loss.
template <bool TRAIN, typename Y>
__global__ void __launch_bounds__(MT)
k_mlp_tile(int B, const float *__restrict__ params, const float *__restrict__ x, const float *__restrict__ t,
           Y *__restrict__ y, float *__restrict__ H1, float *__restrict__ H2, float *__restrict__ GZ1,
           float *__restrict__ GZ2, float *__restrict__ GY, float *__restrict__ loss_part)
{
    __shared__ float s[NPARAM];
    __shared__ float s_w2[NH * PS];
    __shared__ float s_h[MT / 64][RT * PS];         // the wave's H1 tile
    __shared__ float s_g[MT / 64][RT * PS];         // the wave's GZ2 tile
    __shared__ float s_red[MT / 64];
    load_params(params, s);
    for (int e = threadIdx.x; e < NH * NH; e += blockDim.x) s_w2[(e / NH) * PS + e % NH] = params[OW2 + e];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    float *sh = s_h[w], *sg = s_g[w];
    float lsum = 0.f;
    const int tiles = (B + RT - 1) / RT;
    for (int tile = blockIdx.x * (MT / 64) + w; tile < tiles; tile += gridDim.x * (MT / 64)) {
        const int r0 = tile * RT;
        // layer 1: lane a computes column a of the tile's 16 rows
        {
            float wr[NX];
#pragma unroll
            for (int c = 0; c < NX; ++c) wr[c] = s[OW1 + lane * NX + c];
            const float b1 = s[OB1 + lane];
#pragma unroll
            for (int i = 0; i < RT; ++i) {
                const int r = r0 + i;
                float z = b1;
                if (r < B) {
#pragma unroll
                    for (int c = 0; c < NX; ++c) z = fmaf(wr[c], x[(long)r * NX + c], z);
                }
                const float h = r < B ? tanhf(z) : 0.f;
                sh[i * PS + lane] = h;
                if (TRAIN && r < B) H1[(long)r * NH + lane] = h;
            }
        }
        lds_sync_wave();
        // layer 2: Z2 = H1 W2^T, four column blocks of 16
        f4 acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int k4 = 0; k4 < NH; k4 += 4) {
            const int k = k4 + lk;
            const float av = sh[li * PS + k];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = mfma4(av, s_w2[(16 * q + li) * PS + k], acc[q]);
        }
        // bias, tanh, output layer partial sums per row
        float h2v[4][4], yp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * q + li;
                const float h = tanhf(acc[q][r] + s[OB2 + n]);
                h2v[q][r] = h;
                yp[r] = fmaf(s[OW3 + n], h, yp[r]);
                const int row = r0 + 4 * lk + r;
                if (TRAIN && row < B) H2[(long)row * NH + n] = h;
            }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) yp[r] += __shfl_xor(yp[r], o);
        float gyr[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = r0 + 4 * lk + r;
            const float yv = yp[r] + s[OB3];
            gyr[r] = 0.f;
            if (row < B) {
                if (!TRAIN) {
                    if (li == 0) y[row] = (Y)yv;
                } else {
                    const float d = yv - t[row];
                    if (li == 0) {
                        lsum += d * d;
                        GY[row] = 2.f * d / (float)B;
                    }
                    gyr[r] = 2.f * d / (float)B;
                }
            }
        }
        if (TRAIN) {
            // gz2 = gy W3 (1 - h2^2), into the LDS tile and memory
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int n = 16 * q + li, i = 4 * lk + r;
                    const float g = gyr[r] * s[OW3 + n] * (1.f - h2v[q][r] * h2v[q][r]);
                    sg[i * PS + n] = g;
                    if (r0 + i < B) GZ2[(long)(r0 + i) * NH + n] = g;
                }
            lds_sync_wave();
            // GH1 = GZ2 W2, then GZ1 = GH1 (1 - h1^2)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
            for (int k4 = 0; k4 < NH; k4 += 4) {
                const int k = k4 + lk;
                const float av = sg[li * PS + k];
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = mfma4(av, s_w2[k * PS + 16 * q + li], acc[q]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * lk + r, b = 16 * q + li;
                    const float hv = sh[i * PS + b];
                    if (r0 + i < B) GZ1[(long)(r0 + i) * NH + b] = acc[q][r] * (1.f - hv * hv);
                }
        }
        lds_sync_wave();         // the tiles are rewritten by the next tile
    }
    if (TRAIN) {
        for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
        if (lane == 0) s_red[w] = lsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            float tl = 0.f;
            for (int q = 0; q < MT / 64; ++q) tl += s_red[q];
            loss_part[blockIdx.x] = tl / (float)B;
        }
    }
}

// W2 gradient partials: block b sums over its row range (as k_mlp_grad);
// wave w computes output rows a = 16 w .. 16 w + 15 of dW2 = sum_r GZ2[r]^T
// H1[r], four column blocks of 16, K = 4 rows per instruction.
__global__ void __launch_bounds__(MT)
k_mlp_grad_w2(int B, const float *__restrict__ H1, const float *__restrict__ GZ2, float *__restrict__ part)
{
    const int rows_per = (B + gridDim.x - 1) / gridDim.x;
    const int r0 = blockIdx.x * rows_per, r1 = min(B, r0 + rows_per);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    f4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
    for (int rb = r0; rb < r1; rb += 4) {
        const int r = rb + lk;
        const bool ok = r < r1;
        const float av = ok ? GZ2[(long)r * NH + 16 * w + li] : 0.f;     // A[a][row]
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float bv = ok ? H1[(long)r * NH + 16 * q + li] : 0.f;  // B[row][b]
            acc[q] = mfma4(av, bv, acc[q]);
        }
    }
    float *out = part + (size_t)blockIdx.x * NPARAM + OW2;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(16 * w + 4 * lk + r) * NH + 16 * q + li] = acc[q][r];
}

struct TrainWs {
    float *H1, *H2, *GZ1, *GZ2, *GY, *loss_part, *part, *xb, *tb;
    size_t bytes;
};

TrainWs carve(void *base, int B)
{
    TrainWs w{};
    char *p = (char *)base;
    auto take = [&](size_t b) { char *r = p; p += align_up(b, 256); return (float *)r; };
    w.H1 = take(4ull * B * NH);
    w.H2 = take(4ull * B * NH);
    w.GZ1 = take(4ull * B * NH);
    w.GZ2 = take(4ull * B * NH);
    w.GY = take(4ull * B);
    w.loss_part = take(4ull * ((B + RT * (MT / 64) - 1) / (RT * (MT / 64))));
    w.part = take(4ull * GRAD_BLOCKS * NPARAM);
    w.xb = take(4ull * B * NX);
    w.tb = take(4ull * B);
    w.bytes = (size_t)(p - (char *)base);
    return w;
}

}  // namespace
}  // namespace bop

using namespace bop;

extern "C" int bop_features(int n_atoms, int n_orb, int n_max, const double *mu, const float *mean,
                            const float *stdv, float *x, hipStream_t stream)
{
    BOP_REQUIRE(n_atoms >= 0 && n_orb > 0, BOP_E_ARG, "bop_features: bad sizes");
    BOP_REQUIRE(n_max >= NX, BOP_E_ARG, "bop_features: needs n_max >= %d", NX);
    BOP_REQUIRE((mean == nullptr) == (stdv == nullptr), BOP_E_ARG, "bop_features: give both mean and std or neither");
    if (n_atoms == 0) return BOP_OK;
    BOP_REQUIRE(mu && x, BOP_E_ARG, "bop_features: NULL array");
    k_features<<<(n_atoms + 255) / 256, 256, 0, stream>>>(n_atoms, n_orb, n_max, mu, mean, stdv, x);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" int bop_mlp_forward(int n_rows, const float *params, const float *x, float *y, hipStream_t stream)
{
    BOP_REQUIRE(n_rows >= 0, BOP_E_ARG, "bop_mlp_forward: n_rows < 0");
    if (n_rows == 0) return BOP_OK;
    BOP_REQUIRE(params && x && y, BOP_E_ARG, "bop_mlp_forward: NULL array");
    const int tb = (n_rows + RT * (MT / 64) - 1) / (RT * (MT / 64));
    k_mlp_tile<false, float><<<tb, MT, 0, stream>>>(n_rows, params, x, nullptr, y, nullptr, nullptr, nullptr,
                                                   nullptr, nullptr, nullptr);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" int bop_feature_stats(int n_rows, const float *x, float *mean, float *stdv, hipStream_t stream)
{
    BOP_REQUIRE(n_rows > 0, BOP_E_ARG, "bop_feature_stats: n_rows must be > 0");
    BOP_REQUIRE(x && mean && stdv, BOP_E_ARG, "bop_feature_stats: NULL array");
    k_feature_stats<<<NX, MT, 0, stream>>>(n_rows, x, mean, stdv);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" int bop_standardise(int n_rows, const float *x, const float *mean, const float *stdv, float *out,
                               hipStream_t stream)
{
    BOP_REQUIRE(n_rows >= 0, BOP_E_ARG, "bop_standardise: n_rows < 0");
    if (n_rows == 0) return BOP_OK;
    BOP_REQUIRE(x && mean && stdv && out, BOP_E_ARG, "bop_standardise: NULL array");
    const long ne = (long)n_rows * NX;
    k_standardise<<<(unsigned)((ne + 255) / 256), 256, 0, stream>>>(n_rows, x, mean, stdv, out);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" int bop_mlp_shift(int n_rows, const float *params, const float *x, double *shift, hipStream_t stream)
{
    BOP_REQUIRE(n_rows >= 0, BOP_E_ARG, "bop_mlp_shift: n_rows < 0");
    if (n_rows == 0) return BOP_OK;
    BOP_REQUIRE(params && x && shift, BOP_E_ARG, "bop_mlp_shift: NULL array");
    const int tb = (n_rows + RT * (MT / 64) - 1) / (RT * (MT / 64));
    k_mlp_tile<false, double><<<tb, MT, 0, stream>>>(n_rows, params, x, nullptr, shift, nullptr, nullptr, nullptr,
                                                    nullptr, nullptr, nullptr);
    BOP_LAUNCHED();
    k_remove_mean<<<1, 1024, 0, stream>>>(n_rows, shift);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" size_t bop_mlp_train_workspace_size(int batch)
{
    if (batch <= 0) return 0;
    return carve(nullptr, batch).bytes + 256;
}

extern "C" int bop_mlp_train_step(int batch, const int *idx, const float *x, const float *t, float *params,
                                  float *adam_m, float *adam_v, int step, float lr, float *loss, float *grad,
                                  void *ws, size_t ws_bytes, hipStream_t stream)
{
    BOP_REQUIRE(batch > 0 && x && t && params, BOP_E_ARG, "bop_mlp_train_step: bad arguments");
    BOP_REQUIRE(step <= 0 || (adam_m && adam_v), BOP_E_ARG, "bop_mlp_train_step: Adam state NULL");
    TrainWs w = carve(ws, batch);
    BOP_REQUIRE(ws && ws_bytes >= w.bytes, BOP_E_CAPACITY, "bop_mlp_train_step: workspace of %zu bytes needed",
                w.bytes);
    const float *xb = x, *tb = t;
    if (idx) {
        k_gather_rows<<<(batch + 255) / 256, 256, 0, stream>>>(batch, idx, x, t, w.xb, w.tb);
        BOP_LAUNCHED();
        xb = w.xb;
        tb = w.tb;
    }
    const int nfb = (batch + RT * (MT / 64) - 1) / (RT * (MT / 64));
    k_mlp_tile<true, float><<<nfb, MT, 0, stream>>>(batch, params, xb, tb, nullptr, w.H1, w.H2, w.GZ1, w.GZ2, w.GY,
                                                   w.loss_part);
    BOP_LAUNCHED();
    k_mlp_grad<<<GRAD_BLOCKS, MT, 0, stream>>>(batch, xb, w.H1, w.H2, w.GZ1, w.GZ2, w.GY, w.part);
    k_mlp_grad_w2<<<GRAD_BLOCKS, MT, 0, stream>>>(batch, w.H1, w.GZ2, w.part);
    BOP_LAUNCHED();
    k_mlp_adam<<<(NPARAM + AP - 1) / AP, 4 * AP, 0, stream>>>(GRAD_BLOCKS, nfb, w.part, w.loss_part, params, adam_m,
                                                        adam_v, step, lr, grad, loss);
    BOP_LAUNCHED();
    return BOP_OK;
}

extern "C" int bop_mlp_backward(int batch, const int *idx, const float *x, const float *t, const float *params,
                                float *loss, float *grad, void *ws, size_t ws_bytes, hipStream_t stream)
{
    BOP_REQUIRE(grad, BOP_E_ARG, "bop_mlp_backward: grad is NULL");
    // the training step with no update: params are only read
    return bop_mlp_train_step(batch, idx, x, t, const_cast<float *>(params), nullptr, nullptr, 0, 0.f, loss, grad, ws,
                              ws_bytes, stream);
}

extern "C" int bop_mlp_adam(const float *grad, float *params, float *adam_m, float *adam_v, int step, float lr,
                            hipStream_t stream)
{
    BOP_REQUIRE(grad && params && adam_m && adam_v, BOP_E_ARG, "bop_mlp_adam: NULL array");
    BOP_REQUIRE(step >= 1, BOP_E_ARG, "bop_mlp_adam: step must be >= 1");
    k_mlp_adam<<<(NPARAM + AP - 1) / AP, 4 * AP, 0, stream>>>(1, 0, grad, nullptr, params, adam_m, adam_v, step, lr,
                                                        nullptr, nullptr);
    BOP_LAUNCHED();
    return BOP_OK;
}
