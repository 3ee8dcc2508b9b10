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
// Kernels: features (per-atom moment traces, standardised), forward (one row
// per thread, parameters in LDS), and a training step made of a per-row
// forward+backward pass, a per-block gradient reduction over rows, and an
// Adam update that sums the block partials in a fixed order (deterministic).
#include "bop_internal.h"

namespace bop {
namespace {

constexpr int NH = 64, NX = 6;
constexpr int OW1 = 0, OB1 = OW1 + NH * NX, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH, NPARAM = OB3 + 1;
static_assert(NPARAM == BOP_MLP_NPARAM, "parameter count");
constexpr int MT = 256;           // threads per block
constexpr int GRAD_BLOCKS = 128;  // row blocks of the gradient reduction

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

__device__ inline float forward_row(const float *s, const float *xr, float *h1, float *h2)
{
    for (int a = 0; a < NH; ++a) {
        float z = s[OB1 + a];
#pragma unroll
        for (int c = 0; c < NX; ++c) z = fmaf(s[OW1 + a * NX + c], xr[c], z);
        h1[a] = tanhf(z);
    }
    for (int a = 0; a < NH; ++a) {
        float z = s[OB2 + a];
        for (int b = 0; b < NH; ++b) z = fmaf(s[OW2 + a * NH + b], h1[b], z);
        h2[a] = tanhf(z);
    }
    float y = s[OB3];
    for (int b = 0; b < NH; ++b) y = fmaf(s[OW3 + b], h2[b], y);
    return y;
}

template <typename Y>
__global__ void __launch_bounds__(MT)
k_mlp_forward(int n, const float *__restrict__ params, const float *__restrict__ x, Y *__restrict__ y)
{
    __shared__ float s[NPARAM];
    load_params(params, s);
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    float xr[NX], h1[NH], h2[NH];
#pragma unroll
    for (int c = 0; c < NX; ++c) xr[c] = x[(long)r * NX + c];
    y[r] = (Y)forward_row(s, xr, h1, h2);
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

// per row: activations and back-propagated pre-activation gradients
__global__ void __launch_bounds__(MT)
k_mlp_fb(int B, const float *__restrict__ params, const float *__restrict__ x, const float *__restrict__ t,
         float *__restrict__ H1, float *__restrict__ H2, float *__restrict__ GZ1, float *__restrict__ GZ2,
         float *__restrict__ GY, float *__restrict__ loss_part)
{
    __shared__ float s[NPARAM];
    __shared__ float s_red[MT / 64];
    load_params(params, s);
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (r < B) {
        float xr[NX], h1[NH], h2[NH], gz2[NH];
#pragma unroll
        for (int c = 0; c < NX; ++c) xr[c] = x[(long)r * NX + c];
        float y = forward_row(s, xr, h1, h2);
        float d = y - t[r];
        l = d * d;
        float gy = 2.f * d / (float)B;
        GY[r] = gy;
        for (int a = 0; a < NH; ++a) {
            gz2[a] = gy * s[OW3 + a] * (1.f - h2[a] * h2[a]);
            H1[(long)r * NH + a] = h1[a];
            H2[(long)r * NH + a] = h2[a];
            GZ2[(long)r * NH + a] = gz2[a];
        }
        for (int b = 0; b < NH; ++b) {
            float g = 0.f;
            for (int a = 0; a < NH; ++a) g = fmaf(s[OW2 + a * NH + b], gz2[a], g);
            GZ1[(long)r * NH + b] = g * (1.f - h1[b] * h1[b]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        float tl = 0.f;
        for (int w = 0; w < MT / 64; ++w) tl += s_red[w];
        loss_part[blockIdx.x] = tl / (float)B;
    }
}

// partial gradients over one block of rows: every thread owns a strided set
// of parameters and sums its products over the block's rows
__global__ void __launch_bounds__(MT)
k_mlp_grad(int B, const float *__restrict__ x, const float *__restrict__ H1, const float *__restrict__ H2,
           const float *__restrict__ GZ1, const float *__restrict__ GZ2, const float *__restrict__ GY,
           float *__restrict__ part)
{
    const int rows_per = (B + gridDim.x - 1) / gridDim.x;
    const int r0 = blockIdx.x * rows_per, r1 = min(B, r0 + rows_per);
    for (int p = threadIdx.x; p < NPARAM; p += blockDim.x) {
        float g = 0.f;
        if (p < OB1) {
            int a = p / NX, c = p % NX;
            for (int r = r0; r < r1; ++r) g = fmaf(GZ1[(long)r * NH + a], x[(long)r * NX + c], g);
        } else if (p < OW2) {
            int a = p - OB1;
            for (int r = r0; r < r1; ++r) g += GZ1[(long)r * NH + a];
        } else if (p < OB2) {
            int a = (p - OW2) / NH, b = (p - OW2) % NH;
            for (int r = r0; r < r1; ++r) g = fmaf(GZ2[(long)r * NH + a], H1[(long)r * NH + b], g);
        } else if (p < OW3) {
            int a = p - OB2;
            for (int r = r0; r < r1; ++r) g += GZ2[(long)r * NH + a];
        } else if (p < OB3) {
            int b = p - OW3;
            for (int r = r0; r < r1; ++r) g = fmaf(GY[r], H2[(long)r * NH + b], g);
        } else {
            for (int r = r0; r < r1; ++r) g += GY[r];
        }
        part[(size_t)blockIdx.x * NPARAM + p] = g;
    }
}

// sum of the block partials (fixed order) and Adam (lr, 0.9, 0.999, 1e-8)
__global__ void k_mlp_adam(int nblk, int nloss, const float *__restrict__ part, const float *__restrict__ loss_part,
                           float *__restrict__ params, float *__restrict__ m, float *__restrict__ v, int step,
                           float lr, float *__restrict__ grad_out, float *__restrict__ loss)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss) {
        float l = 0.f;
        for (int b = 0; b < nloss; ++b) l += loss_part[b];
        loss[0] = l;
    }
    if (p >= NPARAM) return;
    float g = 0.f;
    for (int b = 0; b < nblk; ++b) g += part[(size_t)b * NPARAM + p];
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
    w.loss_part = take(4ull * ((B + MT - 1) / MT));
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
    k_mlp_forward<float><<<(n_rows + MT - 1) / MT, MT, 0, stream>>>(n_rows, params, x, y);
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
    k_mlp_forward<double><<<(n_rows + MT - 1) / MT, MT, 0, stream>>>(n_rows, params, x, shift);
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
    const int nfb = (batch + MT - 1) / MT;
    k_mlp_fb<<<nfb, MT, 0, stream>>>(batch, params, xb, tb, w.H1, w.H2, w.GZ1, w.GZ2, w.GY, w.loss_part);
    BOP_LAUNCHED();
    k_mlp_grad<<<GRAD_BLOCKS, MT, 0, stream>>>(batch, xb, w.H1, w.H2, w.GZ1, w.GZ2, w.GY, w.part);
    BOP_LAUNCHED();
    k_mlp_adam<<<(NPARAM + 255) / 256, 256, 0, stream>>>(GRAD_BLOCKS, nfb, w.part, w.loss_part, params, adam_m,
                                                        adam_v, step, lr, grad, loss);
    BOP_LAUNCHED();
    return BOP_OK;
}
