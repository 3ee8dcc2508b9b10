// Error reporting and a device-wide exclusive scan shared by the library's
// entry points.
#include "bop_internal.h"

#include <cstring>
#include <mutex>
#include <vector>

namespace bop {

static thread_local char g_err[512];

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

// a device attribute of the current device, cached per (device, slot)
static int cached_attr(int slot, hipDeviceAttribute_t attr, int fallback)
{
    static std::mutex mu;
    static std::vector<int> cache[2];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fallback;
    std::lock_guard<std::mutex> lk(mu);
    std::vector<int> &c = cache[slot];
    if ((int)c.size() <= dev) c.resize(dev + 1, 0);
    if (!c[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, attr, dev) != hipSuccess || v <= 0) v = fallback;
        c[dev] = v;
    }
    return c[dev];
}

int device_cus() { return cached_attr(0, hipDeviceAttributeMultiprocessorCount, 256); }

int device_lds_per_block() { return cached_attr(1, hipDeviceAttributeMaxSharedMemoryPerBlock, 65536); }

// ---------------------------------------------------------------------------
// exclusive scan: 1024 items per block (256 threads x 4), block totals scanned
// recursively, then added back.
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256, SCAN_I = 4, SCAN_CHUNK = SCAN_T * SCAN_I;

__global__ void __launch_bounds__(SCAN_T)
scan_chunks(const int *__restrict__ in, int *__restrict__ out, long n, int *__restrict__ sums)
{
    __shared__ int s[SCAN_T];
    long base = (long)blockIdx.x * SCAN_CHUNK + (long)threadIdx.x * SCAN_I;
    int v[SCAN_I], t = 0;
    for (int k = 0; k < SCAN_I; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        t += v[k];
    }
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int x = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += x;
        __syncthreads();
    }
    int run = s[threadIdx.x] - t;   // exclusive prefix of this thread
    for (int k = 0; k < SCAN_I; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == SCAN_T - 1) sums[blockIdx.x] = s[SCAN_T - 1];
}

__global__ void __launch_bounds__(SCAN_T)
scan_add(int *__restrict__ out, long n, const int *__restrict__ offs)
{
    long base = (long)blockIdx.x * SCAN_CHUNK + (long)threadIdx.x * SCAN_I;
    int o = offs[blockIdx.x];
    for (int k = 0; k < SCAN_I; ++k)
        if (base + k < n) out[base + k] += o;
}

__global__ void scan_total(int *__restrict__ out, long n, const int *__restrict__ in, const int *__restrict__ tot)
{
    // out[n] = out[n-1] + in[n-1]  (n >= 1), or the single-chunk total
    if (n == 0) out[0] = 0;
    else out[n] = tot ? tot[0] : out[n - 1] + in[n - 1];
}

size_t scan_scratch_bytes(long n)
{
    size_t b = 0;
    while (n > 1) {
        long nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
        b += align_up(sizeof(int) * (size_t)(2 * nb + 1), 256);
        n = nb;
    }
    return b + 256;
}

int exclusive_scan(const int *in, int *out, long n, void *scratch, hipStream_t stream)
{
    if (n <= 0) {
        scan_total<<<1, 1, 0, stream>>>(out, 0, in, nullptr);
        BOP_LAUNCHED();
        return BOP_OK;
    }
    long nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    int *sums = (int *)scratch;
    int *offs = sums + nb;
    char *next = (char *)scratch + align_up(sizeof(int) * (size_t)(2 * nb + 1), 256);
    // the last element is needed for the total; read it before `out` may
    // overwrite `in` (in == out is allowed)
    scan_chunks<<<(unsigned)nb, SCAN_T, 0, stream>>>(in, out, n, sums);
    BOP_LAUNCHED();
    if (nb > 1) {
        int rc = exclusive_scan(sums, offs, nb, next, stream);
        if (rc) return rc;
        scan_add<<<(unsigned)nb, SCAN_T, 0, stream>>>(out, n, offs);
        BOP_LAUNCHED();
        scan_total<<<1, 1, 0, stream>>>(out, n, in, offs + nb);
    } else {
        scan_total<<<1, 1, 0, stream>>>(out, n, in, sums);
    }
    BOP_LAUNCHED();
    return BOP_OK;
}

}  // namespace bop

extern "C" int bop_last_error(char *buf, size_t n)
{
    size_t len = strlen(bop::g_err);
    if (buf && n) {
        size_t c = len < n - 1 ? len : n - 1;
        memcpy(buf, bop::g_err, c);
        buf[c] = 0;
    }
    return (int)len;
}
