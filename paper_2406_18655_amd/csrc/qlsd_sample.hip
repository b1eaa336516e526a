// Code-capacity noise on the GPU: Philox4x64-10 uniforms (Salmon et al., SC'11), e_j = [u < p_j],
// s = H e, and logical-failure flags of residuals.  The stream convention is stated in
// include/qlsd_sample.h; every thread computes one Philox block (four consecutive outputs of one
// key), so a shot row's faults come from consecutive counters of its 4096-shot block.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "../../include/qlsd_sample.h"
#include "qlsd_internal.h"

using namespace qlsd;

struct qlsd_sampler_s {
    qlsd_code code;
    DevGraph g;
    double *d_p;       // n
    int k;             // logical rows (0: word error)
    int *d_lrp, *d_lci;
};

namespace {

constexpr int kBlockShots = 4096;

// Published Philox4x64 constants: round multipliers and Weyl key increments.
constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull, kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull, kW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r) { k0 += kW0; k1 += kW1; }
        const uint64_t lo0 = kM0 * c[0], hi0 = __umul64hi(kM0, c[0]);
        const uint64_t lo1 = kM1 * c[2], hi1 = __umul64hi(kM1, c[2]);
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

// One thread per Philox block (4 outputs) of the range's 4096-shot blocks; writes the error bytes
// of the requested shots [start, start + B) that those outputs cover.
__global__ void sample_errors_kernel(const double *p, int n, uint64_t seed, int64_t start, int B, uint8_t *e,
                                     int64_t first_block, int64_t nblocks_words) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t words_per_block = ((int64_t)kBlockShots * n + 3) / 4;
    if (t >= nblocks_words) return;
    const int64_t blk = first_block + t / words_per_block;
    const int64_t w = t % words_per_block;  // counter w + 1 of this block's key
    uint64_t c[4] = {(uint64_t)w + 1ull, 0ull, 0ull, 0ull};
    philox4x64_10(c, seed, (uint64_t)blk);
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int64_t q = 4 * w + u;  // output number inside the block
        const int64_t r = q / n, j = q % n;
        if (r >= kBlockShots) break;
        const int64_t shot = blk * kBlockShots + r - start;
        if (shot < 0 || shot >= B) continue;
        const double x = (double)(c[u] >> 11) * (1.0 / 9007199254740992.0);
        e[shot * n + j] = x < p[j] ? 1 : 0;
    }
}

// s = H x: one thread per (shot, detector), XOR over the detector's CSR row.
__global__ void syndrome_kernel(const int32_t *row_ptr, const int32_t *col_idx, int m, int n, int B,
                                const uint8_t *x, uint8_t *s) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * m) return;
    const int64_t b = t / m;
    const int i = (int)(t % m);
    const uint8_t *row = x + b * n;
    uint8_t acc = 0;
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; e++) acc ^= row[col_idx[e]];
    s[t] = acc & 1;
}

// One wavefront per shot: residual parity against each logical row (or any nonzero fault).
__global__ void failure_kernel(const uint8_t *e, const uint8_t *c, int n, int B, int k, const int *lrp,
                               const int *lci, uint8_t *fail) {
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (b >= B) return;
    const uint8_t *er = e + b * n, *cr = c + b * n;
    bool f = false;
    if (k == 0) {
        bool any = false;
        for (int j = lane; j < n; j += 64) any |= (er[j] ^ cr[j]) & 1;
        f = __ballot(any) != 0ull;
    } else {
        for (int q = 0; q < k && !f; q++) {
            int par = 0;
            for (int x = lrp[q] + lane; x < lrp[q + 1]; x += 64) par ^= (er[lci[x]] ^ cr[lci[x]]) & 1;
            f = (__popcll(__ballot(par != 0)) & 1) != 0;
        }
    }
    if (lane == 0) fail[b] = f ? 1 : 0;
}

qlsd_status sfail(qlsd_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    char buf[256];
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    set_last_error("%s", buf);
    return st;
}

}  // namespace

extern "C" {

qlsd_status qlsd_sampler_create(qlsd_code code, const double *priors, int32_t k, const int32_t *l_row_ptr,
                                const int32_t *l_col_idx, qlsd_sampler *out) {
    set_last_error("");
    if (!out) return sfail(QLSD_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!code || !priors || k < 0 || (k > 0 && (!l_row_ptr || !l_col_idx)))
        return sfail(QLSD_E_INVALID, "NULL code/priors or bad logicals");
    const DevGraph g = code_graph(code);
    for (int j = 0; j < g.n; j++)
        if (!(priors[j] > 0.0 && priors[j] < 1.0)) return sfail(QLSD_E_PRIOR, "prior %d = %g not in (0,1)", j, priors[j]);
    const int nl = k > 0 ? l_row_ptr[k] : 0;
    for (int x = 0; x < nl; x++)
        if (l_col_idx[x] < 0 || l_col_idx[x] >= g.n) return sfail(QLSD_E_INVALID, "logical column out of range");
    qlsd_sampler s = new (std::nothrow) qlsd_sampler_s();
    if (!s) return sfail(QLSD_E_NOMEM, "host allocation failed");
    s->code = code;
    s->g = g;
    s->k = k;
    hipError_t e = hipMalloc((void **)&s->d_p, sizeof(double) * g.n);
    if (e == hipSuccess) e = hipMemcpy(s->d_p, priors, sizeof(double) * g.n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void **)&s->d_lrp, sizeof(int) * (k + 1));
    if (e == hipSuccess && k > 0) e = hipMemcpy(s->d_lrp, l_row_ptr, sizeof(int) * (k + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void **)&s->d_lci, sizeof(int) * (nl > 0 ? nl : 1));
    if (e == hipSuccess && nl > 0) e = hipMemcpy(s->d_lci, l_col_idx, sizeof(int) * nl, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        qlsd_sampler_destroy(s);
        return sfail(QLSD_E_NOMEM, "sampler device allocation failed: %s", hipGetErrorString(e));
    }
    *out = s;
    return QLSD_OK;
}

qlsd_status qlsd_sample(qlsd_sampler s, uint64_t seed, int64_t start, int32_t B, uint8_t *errors,
                        uint8_t *syndromes, void *stream) {
    set_last_error("");
    if (!s || start < 0 || B < 0 || (B > 0 && !errors)) return sfail(QLSD_E_INVALID, "bad sampler call");
    if (B == 0) return QLSD_OK;
    hipStream_t st = (hipStream_t)stream;
    const int n = s->g.n, m = s->g.m;
    const int64_t first = start / kBlockShots, last = (start + B - 1) / kBlockShots;
    const int64_t words = ((int64_t)kBlockShots * n + 3) / 4 * (last - first + 1);
    hipLaunchKernelGGL(sample_errors_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st, s->d_p, n,
                       seed, start, B, errors, first, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return sfail(QLSD_E_DEVICE, "sample launch: %s", hipGetErrorString(e));
    if (syndromes) return qlsd_syndromes(s, errors, B, syndromes, stream);
    (void)m;
    return QLSD_OK;
}

qlsd_status qlsd_syndromes(qlsd_sampler s, const uint8_t *x, int32_t B, uint8_t *syndromes, void *stream) {
    set_last_error("");
    if (!s || B < 0 || (B > 0 && (!x || !syndromes))) return sfail(QLSD_E_INVALID, "bad syndrome call");
    if (B == 0) return QLSD_OK;
    const int64_t total = (int64_t)B * s->g.m;
    hipLaunchKernelGGL(syndrome_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       s->g.row_ptr, s->g.col_idx, s->g.m, s->g.n, B, x, syndromes);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? QLSD_OK : sfail(QLSD_E_DEVICE, "syndrome launch: %s", hipGetErrorString(e));
}

qlsd_status qlsd_failures(qlsd_sampler s, const uint8_t *errors, const uint8_t *corrections, int32_t B,
                          uint8_t *fail, void *stream) {
    set_last_error("");
    if (!s || B < 0 || (B > 0 && (!errors || !corrections || !fail))) return sfail(QLSD_E_INVALID, "bad failure call");
    if (B == 0) return QLSD_OK;
    hipLaunchKernelGGL(failure_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, (hipStream_t)stream, errors,
                       corrections, s->g.n, B, s->k, s->d_lrp, s->d_lci, fail);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? QLSD_OK : sfail(QLSD_E_DEVICE, "failure launch: %s", hipGetErrorString(e));
}

void qlsd_sampler_destroy(qlsd_sampler s) {
    if (!s) return;
    hipFree(s->d_p);
    hipFree(s->d_lrp);
    hipFree(s->d_lci);
    delete s;
}

}  // extern "C"
