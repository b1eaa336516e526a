// Learned reliability refinement between BP and LSD (include/qlsd_net.h): a 3-layer
// message-passing network over the Tanner graph, hidden width 32.  Dense products run on
// bf16 MFMA (v_mfma_f32_16x16x16bf16_1k, float32 accumulate); neighbour means in float32.
// One workgroup (4 wavefronts) per shot at a time; node features of the shot stay in LDS.
// Training keeps the weight-gradient tiles of the nine 32x32 matrices in registers across all
// shots a workgroup processes and adds them to the global gradient once per workgroup.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/qlsd_net.h"
#include "qlsd_internal.h"

namespace qlsd {
namespace {

constexpr int HID = 32;
constexpr int NL = 3;
constexpr int NPAR = QLSD_NET_PARAMS;
constexpr int kNetThreads = 256;
// parameter offsets (floats)
constexpr int P_W0 = 0, P_B0 = 64, P_LAYER = 96, P_LSTRIDE = 3136;
constexpr int P_A = 0, P_a = 1024, P_B = 1056, P_C = 2080, P_b = 3104;
constexpr int P_W = 96 + 3 * 3136, P_BO = P_W + 32;
// small float vectors kept in LDS: W0, b0, a1..3, b1..3, w, bo
constexpr int SV_W0 = 0, SV_B0 = 64, SV_A = 96, SV_BL = 192, SV_W = 288, SV_BO = 320, SV_N = 321;

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));

// float -> bf16, round to nearest even (gfx950 converts in hardware: v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    const float2v v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2v));
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__host__ __device__ inline int pad16(int x) { return (x + 15) & ~15; }
__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

struct NetArgs {
    DevGraph g;
    const float *lam;       // n
    const float *theta;     // NPAR
    const uint8_t *syn;     // B x m
    const float *llr;       // B x n
    const uint8_t *err;     // B x n (training)
    float *llr_out;         // B x n (inference)
    const int *list;        // shots to process (nullable: 0..count-1)
    const int *list_count;  // device count when list != nullptr
    int count;
    float *grad;            // NPAR (training, accumulated)
    float *loss;            // 1 (training, accumulated)
    float inv_total;        // 1 / (shots * n) (training)
    int train;
    unsigned char *act;     // activation workspace, one slice per workgroup (nullptr: in LDS)
    size_t act_stride;      // bytes per slice
    const uint32_t *nbc;    // large-graph inference: [MP][max_rw] byte offsets of fault rows (padded)
    const uint32_t *nbf;    // [NP][max_cw] byte offsets of check rows (padded)
    const float *rdc;       // [MP] 1 / check degree (0 on padding)
    const float *rdf;       // [NP] 1 / fault degree (of the fault in each row)
    const int32_t *perm;    // [NP] large-graph inference: fault held by each feature row (-1: padding)
    const int32_t *tdeg;    // [NP/16] largest fault degree of each 16-row tile
};

struct NetLds {
    int n, m, E, NP, MP;
    uint16_t *wbf;               // 9 x 1024 bf16: [layer][A,B,C][out][in]
    float *sv;                   // small vectors
    float *svg;                  // their gradient accumulators (training)
    uint16_t *rp, *ci, *cp, *ri;
    float *lam, *Lsh;            // n, n
    uint16_t *Hb[NL + 1];        // NP x 32
    uint16_t *Cb[NL + 1];        // MP x 32 (index 1..3)
    uint16_t *AGG;               // max(NP,MP) x 32
    uint16_t *DUV;               // max(NP,MP) x 32 (training)
    float *DH, *DT, *DC;         // NP x 32, max x 32, MP x 32 (training)
    float *misc;                 // [0] loss accumulator
};

// Per-workgroup storage.  The shared part (bf16 weights, small vectors and their gradient
// accumulators, u16 CSR/CSC tables, the loss accumulator) always sits in LDS.  The activation
// part (the shot's BP posteriors, features of every layer, aggregation and backward buffers)
// sits in LDS after it when both fit, else in a workgroup-private slice of a device workspace
// (large graphs such as the 936 x 8800 detector error model); the kernels address both the same way.
__host__ __device__ inline size_t net_shared_layout(int n, int m, int E, bool train, size_t *o) {
    size_t off = 0;
    o[0] = off; off += al16(sizeof(uint16_t) * 9 * 1024);
    o[1] = off; off += al16(sizeof(float) * SV_N);
    o[2] = off; off += train ? al16(sizeof(float) * SV_N) : 0;
    o[3] = off; off += al16(sizeof(uint16_t) * ((size_t)m + 1 + E + n + 1 + E));
    o[4] = off; off += al16(sizeof(float) * 4);
    return off;
}
__host__ __device__ inline size_t net_act_layout(int n, int m, bool train, size_t *o) {
    const int NP = pad16(n), MP = pad16(m), XP = NP > MP ? NP : MP;
    size_t off = 0;
    o[0] = off; off += al16(sizeof(float) * (size_t)n);
    o[1] = off; off += al16(sizeof(uint16_t) * ((NL + 1) * (size_t)NP * HID + NL * (size_t)MP * HID));
    o[2] = off; off += al16(sizeof(uint16_t) * (size_t)XP * HID);
    o[3] = off; off += train ? al16(sizeof(uint16_t) * (size_t)XP * HID) : 0;
    o[4] = off; off += train ? al16(sizeof(float) * ((size_t)NP + XP + MP) * HID) : 0;
    return off;
}

__device__ NetLds carve_net(unsigned char *base, unsigned char *act, int n, int m, int E, bool train,
                            const float *lam) {
    size_t o[5], a5[5];
    net_shared_layout(n, m, E, train, o);
    net_act_layout(n, m, train, a5);
    NetLds L;
    L.n = n; L.m = m; L.E = E; L.NP = pad16(n); L.MP = pad16(m);
    const int XP = L.NP > L.MP ? L.NP : L.MP;
    L.wbf = (uint16_t *)(base + o[0]);
    L.sv = (float *)(base + o[1]);
    L.svg = (float *)(base + o[2]);
    L.rp = (uint16_t *)(base + o[3]);
    L.ci = L.rp + (m + 1);
    L.cp = L.ci + E;
    L.ri = L.cp + (n + 1);
    L.misc = (float *)(base + o[4]);
    L.lam = (float *)lam;
    L.Lsh = (float *)(act + a5[0]);
    uint16_t *a = (uint16_t *)(act + a5[1]);
    for (int l = 0; l <= NL; l++) { L.Hb[l] = a; a += (size_t)L.NP * HID; }
    L.Cb[0] = nullptr;
    for (int l = 1; l <= NL; l++) { L.Cb[l] = a; a += (size_t)L.MP * HID; }
    L.AGG = (uint16_t *)(act + a5[2]);
    L.DUV = (uint16_t *)(act + a5[3]);
    L.DH = (float *)(act + a5[4]);
    L.DT = L.DH + (size_t)L.NP * HID;
    L.DC = L.DT + (size_t)XP * HID;
    return L;
}

// One 16x16 output tile: acc += A[16 x K] * B[K x 16], operands bf16 in LDS addressed by
// strides (element (r,k) of A at A[r*ars + k*aks], element (k,c) of B at B[k*bks + c*bns]).
// Lane layout of v_mfma_f32_16x16x16bf16_1k: lane l supplies A row (l & 15), k = 4(l >> 4)..+3,
// B column (l & 15), same k; it receives D rows 4(l >> 4)..+3 of column (l & 15).
__device__ __forceinline__ float4v mma16(const uint16_t *A, int ars, int aks, const uint16_t *B, int bks, int bns,
                                         int K, float4v acc, int lane) {
    const int r = lane & 15, kq = (lane >> 4) * 4;
    for (int k0 = 0; k0 < K; k0 += 16) {
        short4v a, b;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            a[t] = (short)A[r * ars + (k0 + kq + t) * aks];
            b[t] = (short)B[(k0 + kq + t) * bks + r * bns];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    return acc;
}

__device__ __forceinline__ const uint16_t *Wmat(const NetLds &L, int layer, int which) {  // which: 0 A, 1 B, 2 C
    return L.wbf + ((size_t)(layer - 1) * 3 + which) * 1024;
}

// Mean over the neighbours: dst[node][f] = (1/deg) sum src[nb][f]; rows >= count zero-filled.
__device__ void mean_checks(const NetLds &L, const uint16_t *Hsrc, uint16_t *dst) {  // per check over its faults
    for (int it = threadIdx.x; it < L.MP * HID; it += kNetThreads) {
        const int i = it >> 5, f = it & 31;
        float s = 0.f;
        if (i < L.m) {
            const int e0 = L.rp[i], e1 = L.rp[i + 1];
            for (int e = e0; e < e1; e++) s += bf2f(Hsrc[L.ci[e] * HID + f]);
            if (e1 > e0) s *= 1.0f / (float)(e1 - e0);
        }
        dst[it] = f2bf(s);
    }
}
__device__ void mean_faults(const NetLds &L, const uint16_t *Csrc, uint16_t *dst) {  // per fault over its checks
    for (int it = threadIdx.x; it < L.NP * HID; it += kNetThreads) {
        const int j = it >> 5, f = it & 31;
        float s = 0.f;
        if (j < L.n) {
            const int c0 = L.cp[j], c1 = L.cp[j + 1];
            for (int c = c0; c < c1; c++) s += bf2f(Csrc[L.ri[c] * HID + f]);
            if (c1 > c0) s *= 1.0f / (float)(c1 - c0);
        }
        dst[it] = f2bf(s);
    }
}

// Forward pass of one shot; Hb[0..3], Cb[1..3] hold the activations afterwards.
__device__ void forward_shot(const NetLds &L, const uint8_t *syn, int lane, int wave) {
    // input layer
    for (int it = threadIdx.x; it < L.NP * HID; it += kNetThreads) {
        const int j = it >> 5, f = it & 31;
        float h = 0.f;
        if (j < L.n) {
            const float x0 = tanhf(L.Lsh[j] * 0.125f), x1 = L.lam[j] * 0.125f;
            h = fmaxf(L.sv[SV_W0 + f * 2] * x0 + L.sv[SV_W0 + f * 2 + 1] * x1 + L.sv[SV_B0 + f], 0.f);
        }
        L.Hb[0][it] = f2bf(h);
    }
    __syncthreads();
    for (int l = 1; l <= NL; l++) {
        mean_checks(L, L.Hb[l - 1], L.AGG);
        __syncthreads();
        // c = relu(A m + sigma a)
        for (int tile = wave; tile < (L.MP / 16) * 2; tile += 4) {
            const int rt = tile >> 1, ct = tile & 1;
            float4v acc = {0.f, 0.f, 0.f, 0.f};
            acc = mma16(L.AGG + rt * 16 * HID, HID, 1, Wmat(L, l, 0) + ct * 16 * HID, 1, HID, HID, acc, lane);
            const int col = ct * 16 + (lane & 15);
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const int row = rt * 16 + (lane >> 4) * 4 + t;
                float v = 0.f;
                if (row < L.m) {
                    const float sg = (syn[row] & 1) ? -1.f : 1.f;
                    v = fmaxf(acc[t] + sg * L.sv[SV_A + (l - 1) * HID + col], 0.f);
                }
                L.Cb[l][row * HID + col] = f2bf(v);
            }
        }
        __syncthreads();
        mean_faults(L, L.Cb[l], L.AGG);
        __syncthreads();
        // h = relu(B h + C g + b)
        for (int tile = wave; tile < (L.NP / 16) * 2; tile += 4) {
            const int rt = tile >> 1, ct = tile & 1;
            float4v acc = {0.f, 0.f, 0.f, 0.f};
            acc = mma16(L.Hb[l - 1] + rt * 16 * HID, HID, 1, Wmat(L, l, 1) + ct * 16 * HID, 1, HID, HID, acc, lane);
            acc = mma16(L.AGG + rt * 16 * HID, HID, 1, Wmat(L, l, 2) + ct * 16 * HID, 1, HID, HID, acc, lane);
            const int col = ct * 16 + (lane & 15);
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const int row = rt * 16 + (lane >> 4) * 4 + t;
                const float v = row < L.n ? fmaxf(acc[t] + L.sv[SV_BL + (l - 1) * HID + col], 0.f) : 0.f;
                L.Hb[l][row * HID + col] = f2bf(v);
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ float delta_of(const NetLds &L, int j) {
    float d = L.sv[SV_BO];
    const uint16_t *h = L.Hb[NL] + j * HID;
#pragma unroll
    for (int f = 0; f < HID; f++) d += L.sv[SV_W + f] * bf2f(h[f]);
    return d;
}

__global__ __launch_bounds__(kNetThreads) void net_kernel(NetArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = threadIdx.x;
    const int n = A.g.n, m = A.g.m, E = A.g.nnz;
    const bool train = A.train != 0;
    size_t so[5];
    const size_t shared_bytes = net_shared_layout(n, m, E, train, so);
    unsigned char *act = A.act ? A.act + (size_t)blockIdx.x * A.act_stride : smem + shared_bytes;
    NetLds L = carve_net(smem, act, n, m, E, train, A.lam);

    // weights: 32x32 matrices as bf16, vectors as float
    for (int x = t; x < 9 * 1024; x += kNetThreads) {
        const int mat = x >> 10, layer = mat / 3, which = mat % 3;
        const int off = P_LAYER + layer * P_LSTRIDE + (which == 0 ? P_A : which == 1 ? P_B : P_C) + (x & 1023);
        L.wbf[x] = f2bf(A.theta[off]);
    }
    for (int x = t; x < SV_N; x += kNetThreads) {
        float v;
        if (x < SV_B0) v = A.theta[P_W0 + x];
        else if (x < SV_A) v = A.theta[P_B0 + (x - SV_B0)];
        else if (x < SV_BL) { const int l = (x - SV_A) >> 5; v = A.theta[P_LAYER + l * P_LSTRIDE + P_a + ((x - SV_A) & 31)]; }
        else if (x < SV_W) { const int l = (x - SV_BL) >> 5; v = A.theta[P_LAYER + l * P_LSTRIDE + P_b + ((x - SV_BL) & 31)]; }
        else if (x < SV_BO) v = A.theta[P_W + (x - SV_W)];
        else v = A.theta[P_BO];
        L.sv[x] = v;
        if (train) L.svg[x] = 0.f;
    }
    for (int x = t; x <= m; x += kNetThreads) L.rp[x] = (uint16_t)A.g.row_ptr[x];
    for (int x = t; x < E; x += kNetThreads) L.ci[x] = (uint16_t)A.g.col_idx[x];
    for (int x = t; x <= n; x += kNetThreads) L.cp[x] = (uint16_t)A.g.col_ptr[x];
    for (int x = t; x < E; x += kNetThreads) L.ri[x] = (uint16_t)A.g.row_idx[x];
    if (t == 0) L.misc[0] = 0.f;
    __syncthreads();

    // weight-gradient tiles kept in registers: wavefront w owns tile (w >> 1, w & 1) of each
    // of the nine matrices [layer][A,B,C]
    float4v gacc[9];
#pragma unroll
    for (int q = 0; q < 9; q++) gacc[q] = (float4v){0.f, 0.f, 0.f, 0.f};
    const int trow = (wave >> 1) * 16, tcol = (wave & 1) * 16;

    const int total = A.list ? *A.list_count : A.count;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int shot = A.list ? A.list[item] : item;
        const uint8_t *syn = A.syn + (size_t)shot * m;
        const float *llr = A.llr + (size_t)shot * n;
        for (int j = t; j < n; j += kNetThreads) L.Lsh[j] = llr[j];
        __syncthreads();
        forward_shot(L, syn, lane, wave);

        if (!train) {
            for (int j = t; j < n; j += kNetThreads) A.llr_out[(size_t)shot * n + j] = L.Lsh[j] + delta_of(L, j);
            __syncthreads();
            continue;
        }

        // ---- loss and output layer
        const uint8_t *err = A.err + (size_t)shot * n;
        for (int it = t; it < L.NP * HID; it += kNetThreads) L.DH[it] = 0.f;
        __syncthreads();
        for (int j = t; j < n; j += kNetThreads) {
            const float Lp = L.Lsh[j] + delta_of(L, j);
            const float e = (float)(err[j] & 1);
            // softplus(-L') + e L'
            const float lossj = fmaxf(-Lp, 0.f) + log1pf(expf(-fabsf(Lp))) + e * Lp;
            atomicAdd(&L.misc[0], lossj * A.inv_total);
            const float dD = (e - 1.f / (1.f + expf(Lp))) * A.inv_total;
            atomicAdd(&L.svg[SV_BO], dD);
            const uint16_t *h = L.Hb[NL] + j * HID;
            for (int f = 0; f < HID; f++) {
                atomicAdd(&L.svg[SV_W + f], dD * bf2f(h[f]));
                L.DH[j * HID + f] = dD * L.sv[SV_W + f];
            }
        }
        __syncthreads();
        for (int l = NL; l >= 1; l--) {
            // du = dh * [h_l > 0]; db_l; g_l recomputed into AGG
            for (int it = t; it < L.NP * HID; it += kNetThreads) {
                const float du = bf2f(L.Hb[l][it]) > 0.f ? L.DH[it] : 0.f;
                L.DUV[it] = f2bf(du);
                if (du != 0.f) atomicAdd(&L.svg[SV_BL + (l - 1) * HID + (it & 31)], du);
            }
            mean_faults(L, L.Cb[l], L.AGG);
            __syncthreads();
            // dB += du^T h_{l-1}, dC += du^T g  (K = faults)
            gacc[(l - 1) * 3 + 1] = mma16(L.DUV + trow, 1, HID, L.Hb[l - 1] + tcol, HID, 1, L.NP,
                                          gacc[(l - 1) * 3 + 1], lane);
            gacc[(l - 1) * 3 + 2] = mma16(L.DUV + trow, 1, HID, L.AGG + tcol, HID, 1, L.NP, gacc[(l - 1) * 3 + 2], lane);
            // dg = du C -> DT, dh_{l-1} = du B -> DH
            for (int tile = wave; tile < (L.NP / 16) * 4; tile += 4) {
                const int rt = tile >> 2, which = (tile >> 1) & 1, ct = tile & 1;
                float4v acc = {0.f, 0.f, 0.f, 0.f};
                acc = mma16(L.DUV + rt * 16 * HID, HID, 1, Wmat(L, l, which == 0 ? 2 : 1) + ct * 16, HID, 1, HID, acc,
                            lane);
                float *dst = which == 0 ? L.DT : L.DH;
                const int col = ct * 16 + (lane & 15);
#pragma unroll
                for (int q = 0; q < 4; q++) dst[(rt * 16 + (lane >> 4) * 4 + q) * HID + col] = acc[q];
            }
            __syncthreads();
            // dc_i = sum_{j in N(i)} dg_j / deg_j
            for (int it = t; it < L.MP * HID; it += kNetThreads) {
                const int i = it >> 5, f = it & 31;
                float s = 0.f;
                if (i < m) {
                    for (int e = L.rp[i]; e < L.rp[i + 1]; e++) {
                        const int j = L.ci[e];
                        s += L.DT[j * HID + f] / (float)(L.cp[j + 1] - L.cp[j]);
                    }
                }
                L.DC[it] = s;
            }
            __syncthreads();
            // dv = dc * [c > 0]; da; m_l recomputed into AGG
            for (int it = t; it < L.MP * HID; it += kNetThreads) {
                const int i = it >> 5;
                const float dv = bf2f(L.Cb[l][it]) > 0.f ? L.DC[it] : 0.f;
                L.DUV[it] = f2bf(dv);
                if (dv != 0.f) atomicAdd(&L.svg[SV_A + (l - 1) * HID + (it & 31)], (syn[i] & 1) ? -dv : dv);
            }
            mean_checks(L, L.Hb[l - 1], L.AGG);
            __syncthreads();
            // dA += dv^T m (K = checks); dm = dv A -> DT
            gacc[(l - 1) * 3 + 0] = mma16(L.DUV + trow, 1, HID, L.AGG + tcol, HID, 1, L.MP, gacc[(l - 1) * 3 + 0], lane);
            for (int tile = wave; tile < (L.MP / 16) * 2; tile += 4) {
                const int rt = tile >> 1, ct = tile & 1;
                float4v acc = {0.f, 0.f, 0.f, 0.f};
                acc = mma16(L.DUV + rt * 16 * HID, HID, 1, Wmat(L, l, 0) + ct * 16, HID, 1, HID, acc, lane);
                const int col = ct * 16 + (lane & 15);
#pragma unroll
                for (int q = 0; q < 4; q++) L.DT[(rt * 16 + (lane >> 4) * 4 + q) * HID + col] = acc[q];
            }
            __syncthreads();
            // dh_{l-1} += sum_{i in N(j)} dm_i / deg_i
            for (int it = t; it < L.NP * HID; it += kNetThreads) {
                const int j = it >> 5, f = it & 31;
                if (j < n) {
                    float s = 0.f;
                    for (int c = L.cp[j]; c < L.cp[j + 1]; c++) {
                        const int i = L.ri[c];
                        s += L.DT[i * HID + f] / (float)(L.rp[i + 1] - L.rp[i]);
                    }
                    L.DH[it] += s;
                }
            }
            __syncthreads();
        }
        // input layer
        for (int it = t; it < n * HID; it += kNetThreads) {
            const int j = it >> 5, f = it & 31;
            if (bf2f(L.Hb[0][it]) > 0.f) {
                const float du = L.DH[it];
                const float x0 = tanhf(L.Lsh[j] * 0.125f), x1 = L.lam[j] * 0.125f;
                atomicAdd(&L.svg[SV_W0 + f * 2], du * x0);
                atomicAdd(&L.svg[SV_W0 + f * 2 + 1], du * x1);
                atomicAdd(&L.svg[SV_B0 + f], du);
            }
        }
        __syncthreads();
    }
    if (!train) return;
    // flush: matrix tiles (acc rows = out feature, cols = in feature), vectors, loss
#pragma unroll
    for (int q = 0; q < 9; q++) {
        const int layer = q / 3, which = q % 3;
        const int base = P_LAYER + layer * P_LSTRIDE + (which == 0 ? P_A : which == 1 ? P_B : P_C);
        const int col = tcol + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int row = trow + (lane >> 4) * 4 + r;
            atomicAdd(&A.grad[base + row * HID + col], gacc[q][r]);
        }
    }
    __syncthreads();
    for (int x = t; x < SV_N; x += kNetThreads) {
        int off;
        if (x < SV_B0) off = P_W0 + x;
        else if (x < SV_A) off = P_B0 + (x - SV_B0);
        else if (x < SV_BL) off = P_LAYER + ((x - SV_A) >> 5) * P_LSTRIDE + P_a + ((x - SV_A) & 31);
        else if (x < SV_W) off = P_LAYER + ((x - SV_BL) >> 5) * P_LSTRIDE + P_b + ((x - SV_BL) & 31);
        else if (x < SV_BO) off = P_W + (x - SV_W);
        else off = P_BO;
        atomicAdd(&A.grad[off], L.svg[x]);
    }
    if (t == 0) atomicAdd(A.loss, L.misc[0]);
}


// ------------------------------------------------------------------------------------------
// Inference: one wavefront per shot, no workgroup barriers.  The A/B/C weight fragments of all
// three layers sit in registers (9 matrices x 2 output tiles of 8 bf16 per lane), and each
// product covers the whole hidden width in one v_mfma_f32_16x16x32_bf16 (gfx950's double-K form,
// twice the rate of the 16x16x16 form per issued instruction).
// Products are formed transposed, D = W X^T, with the output rows of W permuted so that after
// the two products of a layer (two 16-feature output tiles) a lane holds 8 consecutive output
// features of one node -- the same feature group the next product reads -- and results leave
// as one packed 16-byte word.  The neighbour means enter by linearity,
//     A m_i = (1/deg_i) sum_{j in N(i)} A h_j,     C g_j = (1/deg_j) sum_{i in N(j)} C c_i,
// so each neighbour's bf16 feature words feed the MFMA directly (no unpacking or vector sums)
// and the 1/deg scaling is applied to the float32 accumulator.  Neighbour lists are padded to
// the maximum degree with a zero sentinel row.  Compared with forward_shot (the training
// forward) the means are not rounded to bf16 before the product; everything else matches.
// ------------------------------------------------------------------------------------------
constexpr int kInferWavesMax = 11;  // one workgroup of up to 11 wavefronts per CU, else 5 (two per CU)

__host__ __device__ inline size_t infer_shared_bytes(int n, int m, int dr, int dc) {
    return al16(sizeof(float) * SV_N) + al16(sizeof(uint16_t) * ((size_t)pad16(m) * dr + (size_t)pad16(n) * dc)) +
           al16(sizeof(float) * ((size_t)pad16(m) + pad16(n) + n));
}
// Per wavefront: fault and check feature rows (bf16 x 32 each), plus one zero sentinel row each
// for the padding of irregular neighbour lists (a code with every row and every column of full
// weight pads nothing but its 16-row tiles, whose results are discarded), and one signed byte
// per check of the padded tiles for the syndrome sign (0 on padding).
__host__ __device__ inline bool infer_regular(const DevGraph &g) {
    return g.min_rw == g.max_rw && g.min_cw == g.max_cw;
}
__host__ __device__ inline size_t infer_wave_bytes(int n, int m, bool regular) {
    return al16(sizeof(uint16_t) * ((size_t)pad16(n) + pad16(m) + (regular ? 0 : 2)) * HID) + al16((size_t)pad16(m));
}

// Feature rows are 64 B: 32 bf16 as four 16-byte groups of 8 features.  Group q of node v sits at
// group position q ^ f(v), f(v) = ((v >> 1) & 3) ^ ((v >> 3) & 1), of its row.  Over 16 consecutive
// nodes (a tile) and a fixed group, any 8 aligned nodes then cover all 8 16-byte slots of a
// 128-byte bank window and any 4 nodes equal mod 4 all 4 slots of their 64-byte quarter of a
// 256-byte window, so the tile's 16-byte reads and writes are free of bank conflicts with either
// width of LDS bank set.  The swizzled row offset srow(v) = 64 v | (f(v) << 4) carries the
// swizzle: group q of node v is at srow(v) ^ 16 q, and the neighbour tables hold srow() of each
// neighbour, so a gather costs one XOR per load.  f depends on bits 1..3 of v only, so the row
// of node 16 rt + r sits at 1024 rt + srow(r).
__host__ __device__ __forceinline__ int srow(int node) {
    return node * 64 | ((((node >> 1) & 3) ^ ((node >> 3) & 1)) << 4);
}
// Features 8q .. 8q+7 of the node with swizzled row offset so: the operand a lane of group q
// supplies to v_mfma_f32_16x16x32_bf16 (lane l: column l & 15, k = 8 (l >> 4) .. +7).
__device__ __forceinline__ bf16x8v lds_group(const unsigned char *base, int so, int q16) {
    return *(const bf16x8v *)(base + (so ^ q16));
}
__device__ __forceinline__ float4v mfma32(bf16x8v a, bf16x8v b, float4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int DR, int DC>
__global__ __launch_bounds__(64 * kInferWavesMax) void net_infer_kernel(NetArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = threadIdx.x;
    const int n = A.g.n, m = A.g.m, NP = pad16(n), MP = pad16(m);
    const int dr = DR ? DR : A.g.max_rw, dc = DC ? DC : A.g.max_cw;
    float *sv = (float *)smem;
    uint16_t *nbc = (uint16_t *)(smem + al16(sizeof(float) * SV_N));  // [MP][dr] byte offsets into H
    uint16_t *nbf = nbc + (size_t)MP * dr;                             // [NP][dc] byte offsets into C
    float *rdc = (float *)((unsigned char *)nbc + al16(sizeof(uint16_t) * ((size_t)MP * dr + (size_t)NP * dc)));
    float *rdf = rdc + MP, *lam = rdf + NP;
    const bool reg = infer_regular(A.g);
    const int nwav = blockDim.x >> 6;
    unsigned char *wbase = smem + infer_shared_bytes(n, m, dr, dc) + (size_t)wave * infer_wave_bytes(n, m, reg);
    const int sent = reg ? 0 : 1;                    // sentinel rows present
    uint16_t *H = (uint16_t *)wbase;                 // (NP + sent) x 32, row NP (if present) is zero
    uint16_t *Cf = H + (size_t)(NP + sent) * HID;    // (MP + sent) x 32, row MP (if present) is zero
    int8_t *sg = (int8_t *)(wbase + al16(sizeof(uint16_t) * ((size_t)NP + MP + 2 * sent) * HID));  // +-1 per check
    unsigned char *Hb = (unsigned char *)H, *Cb = (unsigned char *)Cf;

    for (int x = t; x < SV_N; x += blockDim.x) {
        float v;
        if (x < SV_B0) v = A.theta[P_W0 + x];
        else if (x < SV_A) v = A.theta[P_B0 + (x - SV_B0)];
        else if (x < SV_BL) { const int l = (x - SV_A) >> 5; v = A.theta[P_LAYER + l * P_LSTRIDE + P_a + ((x - SV_A) & 31)]; }
        else if (x < SV_W) { const int l = (x - SV_BL) >> 5; v = A.theta[P_LAYER + l * P_LSTRIDE + P_b + ((x - SV_BL) & 31)]; }
        else if (x < SV_BO) v = A.theta[P_W + (x - SV_W)];
        else v = A.theta[P_BO];
        sv[x] = v;
    }
    for (int x = t; x < MP * dr; x += blockDim.x) {
        const int i = x / dr, k = x - i * dr;
        int v = sent * NP;
        if (i < m) {
            const int e0 = A.g.row_ptr[i], e1 = A.g.row_ptr[i + 1];
            if (e0 + k < e1) v = A.g.col_idx[e0 + k];
        }
        nbc[x] = (uint16_t)srow(v);
    }
    for (int x = t; x < NP * dc; x += blockDim.x) {
        const int j = x / dc, k = x - j * dc;
        int v = sent * MP;
        if (j < n) {
            const int c0 = A.g.col_ptr[j], c1 = A.g.col_ptr[j + 1];
            if (c0 + k < c1) v = A.g.row_idx[c0 + k];
        }
        nbf[x] = (uint16_t)srow(v);
    }
    for (int x = t; x < MP; x += blockDim.x) {
        const int d = x < m ? A.g.row_ptr[x + 1] - A.g.row_ptr[x] : 0;
        rdc[x] = d > 0 ? 1.0f / (float)d : 0.f;
    }
    for (int x = t; x < NP; x += blockDim.x) {
        const int d = x < n ? A.g.col_ptr[x + 1] - A.g.col_ptr[x] : 0;
        rdf[x] = d > 0 ? 1.0f / (float)d : 0.f;
        if (x < n) lam[x] = A.lam[x];
    }
    // sentinel rows (never written again)
    if (sent && lane < 16) {
        ((uint32_t *)(H + (size_t)NP * HID))[lane] = 0u;
        ((uint32_t *)(Cf + (size_t)MP * HID))[lane] = 0u;
    }
    __syncthreads();

    // A-operand fragments of v_mfma_f32_16x16x32_bf16 (the whole hidden width in one product).
    // Output tile ot's row r computes feature 8 (r >> 2) + 4 ot + (r & 3), so that the lane
    // holding rows 4 q8 .. +3 of both tiles holds features 8 q8 .. 8 q8 + 7: one whole feature
    // group, stored as one 16-byte word.  wf[mat][ot] = W[8 (r16 >> 2) + 4 ot + (r16 & 3)][8 q8 .. +7]
    const int r16 = lane & 15, q8 = lane >> 4;
    bf16x8v wf[9][2];
#pragma unroll
    for (int mat = 0; mat < 9; mat++) {
        const int layer = mat / 3, which = mat % 3;
        const float *W = A.theta + P_LAYER + layer * P_LSTRIDE + (which == 0 ? P_A : which == 1 ? P_B : P_C);
#pragma unroll
        for (int ot = 0; ot < 2; ot++) {
            const float *w = W + (8 * (r16 >> 2) + 4 * ot + (r16 & 3)) * HID + 8 * q8;
            wf[mat][ot] = __builtin_bit_cast(bf16x8v, make_uint4(pack_bf16x2(w[0], w[1]), pack_bf16x2(w[2], w[3]),
                                                                pack_bf16x2(w[4], w[5]), pack_bf16x2(w[6], w[7])));
        }
    }

    // per lane: the tile row's swizzled offset is 1024 rt + srow(lane & 15), and the lane reads,
    // and after a product writes, feature group q8 of that row (byte offset go within the tile)
    const int q16 = q8 << 4, go = srow(r16) ^ q16;
    const int total = A.list ? *A.list_count : A.count;
    for (int item = blockIdx.x * nwav + wave; item < total; item += gridDim.x * nwav) {
        const int shot = A.list ? A.list[item] : item;
        const uint8_t *syn = A.syn + (size_t)shot * m;
        const float *llr = A.llr + (size_t)shot * n;
        for (int i = lane; i < MP; i += 64) sg[i] = i < m ? ((syn[i] & 1) ? -1 : 1) : 0;
        // input layer: lane j computes tanh once and writes its fault's 32 features (4 x 16 B).
        // Padding nodes (j >= n) get relu(b0): no neighbour list names them and no output reads them.
        for (int j = lane; j < NP; j += 64) {
            float x0 = 0.f, x1 = 0.f;
            if (j < n) { x0 = tanhf(llr[j] * 0.125f); x1 = lam[j] * 0.125f; }
            const int so = srow(j);
#pragma unroll
            for (int f8 = 0; f8 < HID; f8 += 8) {
                uint32_t w[4];
#pragma unroll
                for (int h2 = 0; h2 < 4; h2++) {
                    const int f = f8 + 2 * h2;
                    const float v0 = fmaxf(sv[SV_W0 + f * 2] * x0 + sv[SV_W0 + f * 2 + 1] * x1 + sv[SV_B0 + f], 0.f);
                    const float v1 = fmaxf(sv[SV_W0 + f * 2 + 2] * x0 + sv[SV_W0 + f * 2 + 3] * x1 + sv[SV_B0 + f + 1], 0.f);
                    w[h2] = pack_bf16x2(v0, v1);
                }
                *(uint4 *)(Hb + (so ^ ((f8 >> 3) << 4))) = make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int l = 0; l < NL; l++) {
            // checks: c_i = relu((1/deg_i) sum_j A h_j + sigma_i a)
            for (int rt = 0; rt < MP / 16; rt++) {
                const int i = rt * 16 + r16;
                float4v acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
                const uint16_t *nb = nbc + i * dr;
#pragma unroll
                for (int k = 0; k < (DR ? DR : dr); k++) {
                    const bf16x8v x = lds_group(Hb, nb[k], q16);
#pragma unroll
                    for (int ot = 0; ot < 2; ot++) acc[ot] = mfma32(wf[l * 3 + 0][ot], x, acc[ot]);
                }
                const float rd = rdc[i], sgn = (float)sg[i];
                uint32_t w[4];
#pragma unroll
                for (int ot = 0; ot < 2; ot++) {
                    const float4v av = *(const float4v *)(sv + SV_A + l * HID + 8 * q8 + 4 * ot);
                    float v[4];
#pragma unroll
                    for (int q = 0; q < 4; q++) v[q] = fmaxf(rd * acc[ot][q] + sgn * av[q], 0.f);
                    w[2 * ot] = pack_bf16x2(v[0], v[1]);
                    w[2 * ot + 1] = pack_bf16x2(v[2], v[3]);
                }
                *(uint4 *)(Cb + rt * 1024 + go) = make_uint4(w[0], w[1], w[2], w[3]);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // faults: h_j = relu(B h_j + b + (1/deg_j) sum_i C c_i), b entering as the accumulator of
            // B h_j (in place: a lane reads and writes only its own node's words; padding rows
            // are computed like the rest and never read)
            for (int rt = 0; rt < NP / 16; rt++) {
                const int j = rt * 16 + r16;
                const bf16x8v h = *(const bf16x8v *)(Hb + rt * 1024 + go);
                float4v as[2], an[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
                for (int ot = 0; ot < 2; ot++)
                    as[ot] = mfma32(wf[l * 3 + 1][ot], h, *(const float4v *)(sv + SV_BL + l * HID + 8 * q8 + 4 * ot));
                const uint16_t *nb = nbf + j * dc;
#pragma unroll
                for (int k = 0; k < (DC ? DC : dc); k++) {
                    const bf16x8v y = lds_group(Cb, nb[k], q16);
#pragma unroll
                    for (int ot = 0; ot < 2; ot++) an[ot] = mfma32(wf[l * 3 + 2][ot], y, an[ot]);
                }
                const float rd = rdf[j];
                uint32_t w[4];
#pragma unroll
                for (int ot = 0; ot < 2; ot++) {
                    float v[4];
#pragma unroll
                    for (int q = 0; q < 4; q++) v[q] = fmaxf(rd * an[ot][q] + as[ot][q], 0.f);
                    w[2 * ot] = pack_bf16x2(v[0], v[1]);
                    w[2 * ot + 1] = pack_bf16x2(v[2], v[3]);
                }
                *(uint4 *)(Hb + rt * 1024 + go) = make_uint4(w[0], w[1], w[2], w[3]);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        for (int j = lane; j < n; j += 64) {
            float d = sv[SV_BO];
            const int so = srow(j);
#pragma unroll
            for (int f8 = 0; f8 < 4; f8++) {
                const uint4 v = *(const uint4 *)(Hb + (so ^ (f8 << 4)));
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int h2 = 0; h2 < 4; h2++) {
                    d += sv[SV_W + f8 * 8 + 2 * h2] * __uint_as_float(w[h2] << 16);
                    d += sv[SV_W + f8 * 8 + 2 * h2 + 1] * __uint_as_float(w[h2] & 0xffff0000u);
                }
            }
            A.llr_out[(size_t)shot * n + j] = llr[j] + d;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}


// ------------------------------------------------------------------------------------------
// Large-graph inference (graphs whose features do not fit in LDS, e.g. the 936 x 8800 detector
// error model): one workgroup per shot, its wavefronts splitting the 16-node tiles of each
// phase, features in a workgroup-private slice of the device workspace (kept in the last-level
// cache across the grid).  The arithmetic is that of net_infer_kernel: transposed products on
// v_mfma_f32_16x16x32_bf16 with the output rows of W permuted so that a lane ends a layer holding
// one whole 8-feature group (one 16-byte store), neighbour means by linearity on the float32
// accumulator, zero sentinel rows for padding.  Fault rows are stored sorted by degree (row r
// holds fault perm[r]), so the 16 faults of a tile have equal or near-equal degree and a tile
// gathers only up to its own largest degree (tdeg[tile]) instead of the code's; the network
// treats every node alike and each neighbour sum keeps its order, so the row order changes no
// result.  The fault phase issues the loads of two tiles before their products; the check
// phase loads the next group's table entries while the current group's gathers are in flight.
// The input layer is never stored: layer 0 recomputes a fault's first-layer features from its
// 8-byte inputs (tanh(L/8), lambda/8) where it needs them, and the last fault phase applies the
// output layer to its own bf16-rounded features instead of storing them.
// ------------------------------------------------------------------------------------------
constexpr int kBigWaves = 16;
constexpr int kGather = 10;      // check-phase gathers in flight per tile
constexpr int kFaultGather = 6;  // fault-phase gathers per tile and pass (heavier tiles loop)
constexpr int kFaultTiles = 2;   // fault tiles per pass

// Fault row order of the large-graph kernel: faults sorted by degree, largest first (stable);
// rows n .. pad16(n)-1 are padding (-1).
static void big_fault_order(const std::vector<int32_t> &col_ptr, int n, std::vector<int32_t> &perm,
                            std::vector<int32_t> &rowof, std::vector<int32_t> &tdeg) {
    const int NP = pad16(n);
    int maxd = 0;
    for (int j = 0; j < n; j++) maxd = std::max(maxd, col_ptr[j + 1] - col_ptr[j]);
    std::vector<int> start(maxd + 2, 0);
    for (int j = 0; j < n; j++) start[maxd - (col_ptr[j + 1] - col_ptr[j]) + 1]++;
    for (int d = 1; d <= maxd + 1; d++) start[d] += start[d - 1];
    perm.assign(NP, -1);
    rowof.assign(n, 0);
    for (int j = 0; j < n; j++) {
        const int r = start[maxd - (col_ptr[j + 1] - col_ptr[j])]++;
        perm[r] = j;
        rowof[j] = r;
    }
    tdeg.assign(NP / 16, 0);
    for (int r = 0; r < n; r++) {
        const int j = perm[r];
        tdeg[r >> 4] = std::max(tdeg[r >> 4], col_ptr[j + 1] - col_ptr[j]);
    }
}

__global__ void big_tables_kernel(DevGraph g, const int32_t *perm, const int32_t *rowof, uint32_t *nbc, uint32_t *nbf,
                                  float *rdc, float *rdf) {
    const int NP = pad16(g.n), MP = pad16(g.m), dr = g.max_rw, dc = g.max_cw;
    const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t x = tid; x < (size_t)MP * dr; x += stride) {
        const int i = (int)(x / dr), k = (int)(x % dr);
        uint32_t off = (uint32_t)NP * 64u;
        if (i < g.m && g.row_ptr[i] + k < g.row_ptr[i + 1]) off = (uint32_t)rowof[g.col_idx[g.row_ptr[i] + k]] * 64u;
        nbc[x] = off;
    }
    for (size_t x = tid; x < (size_t)NP * dc; x += stride) {
        const int r = (int)(x / dc), k = (int)(x % dc), j = perm[r];
        uint32_t off = (uint32_t)MP * 64u;
        if (j >= 0 && g.col_ptr[j] + k < g.col_ptr[j + 1]) off = (uint32_t)g.row_idx[g.col_ptr[j] + k] * 64u;
        nbf[x] = off;
    }
    for (size_t x = tid; x < (size_t)MP; x += stride) {
        const int d = x < (size_t)g.m ? g.row_ptr[x + 1] - g.row_ptr[x] : 0;
        rdc[x] = d > 0 ? 1.0f / (float)d : 0.f;
    }
    for (size_t x = tid; x < (size_t)NP; x += stride) {
        const int j = perm[x];
        const int d = j >= 0 ? g.col_ptr[j + 1] - g.col_ptr[j] : 0;
        rdf[x] = d > 0 ? 1.0f / (float)d : 0.f;
    }
}

// dynamic LDS of net_infer_big_kernel: syndrome signs and the u16 fault neighbour table (the
// kernel also holds 20 KB of static LDS)
__host__ __device__ inline size_t big_dyn_lds(const DevGraph &g) {
    return al16(sizeof(float) * (size_t)g.m) + al16(sizeof(uint16_t) * (size_t)pad16(g.n) * g.max_cw);
}
// per-workgroup slice: fault rows (NP + 1 with the zero row), check rows (MP + 1), and each fault
// row's inputs (x0, x1) as a float pair (NP + 1: the zero row's entry is read, then discarded)
__host__ __device__ inline size_t big_slice_bytes(int n, int m) {
    return al16(sizeof(uint16_t) * ((size_t)pad16(n) + 1 + pad16(m) + 1) * HID) +
           al16(sizeof(float) * 2 * ((size_t)pad16(n) + 1));
}

__device__ __forceinline__ bf16x8v gload(const unsigned char *base, uint32_t off) {
    return *(const bf16x8v *)(base + off);
}

__global__ __launch_bounds__(64 * kBigWaves) void net_infer_big_kernel(NetArgs A) {
    __shared__ __align__(16) float sv[SV_N];
    __shared__ uint4 wfl[9 * 2 * 64];  // weight fragments [mat][ot][lane], output rows permuted
    extern __shared__ __align__(16) unsigned char smem[];  // sg: m floats; then fault neighbour rows
    const int lane = threadIdx.x & 63, t = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = A.g.n, m = A.g.m, NP = pad16(n), MP = pad16(m), dr = A.g.max_rw, dc = A.g.max_cw;
    float *sg = (float *)smem;
    // the fault phase's neighbour lists as u16 check rows (MP = the zero row), read from LDS
    uint16_t *nbf16 = (uint16_t *)(smem + al16(sizeof(float) * (size_t)m));
    for (int x = t; x < NP * dc; x += blockDim.x) nbf16[x] = (uint16_t)(A.nbf[x] >> 6);
    unsigned char *Hb = A.act + (size_t)blockIdx.x * A.act_stride;
    unsigned char *Cb = Hb + (size_t)(NP + 1) * 64;

    for (int x = t; x < SV_N; x += blockDim.x) {
        float v;
        if (x < SV_B0) v = A.theta[P_W0 + x];
        else if (x < SV_A) v = A.theta[P_B0 + (x - SV_B0)];
        else if (x < SV_BL) { const int l = (x - SV_A) >> 5; v = A.theta[P_LAYER + l * P_LSTRIDE + P_a + ((x - SV_A) & 31)]; }
        else if (x < SV_W) { const int l = (x - SV_BL) >> 5; v = A.theta[P_LAYER + l * P_LSTRIDE + P_b + ((x - SV_BL) & 31)]; }
        else if (x < SV_BO) v = A.theta[P_W + (x - SV_W)];
        else v = A.theta[P_BO];
        sv[x] = v;
    }
    // A-operand fragment (mat, ot) of lane l: W[8 (r >> 2) + 4 ot + (r & 3)][8 q .. 8 q + 7], r = l & 15,
    // q = l >> 4 (the output-row order of net_infer_kernel)
    for (int x = t; x < 9 * 2 * 64; x += blockDim.x) {
        const int l = x & 63, ot = (x >> 6) & 1, mat = x >> 7;
        const int layer = mat / 3, which = mat % 3, r = l & 15, q = l >> 4;
        const float *W = A.theta + P_LAYER + layer * P_LSTRIDE + (which == 0 ? P_A : which == 1 ? P_B : P_C);
        const float *w = W + (8 * (r >> 2) + 4 * ot + (r & 3)) * HID + 8 * q;
        wfl[x] = make_uint4(pack_bf16x2(w[0], w[1]), pack_bf16x2(w[2], w[3]), pack_bf16x2(w[4], w[5]),
                            pack_bf16x2(w[6], w[7]));
    }
    if (t < 16) {  // sentinel rows (never written again)
        ((uint32_t *)(Hb + (size_t)NP * 64))[t] = 0u;
        ((uint32_t *)(Cb + (size_t)MP * 64))[t] = 0u;
    }
    const int r16 = lane & 15, q8 = lane >> 4, q16 = q8 << 4;
    __syncthreads();
    auto frag = [&](int mat, int ot) { return __builtin_bit_cast(bf16x8v, wfl[(mat * 2 + ot) * 64 + lane]); };
    auto store_group = [&](unsigned char *p, const float4v &v0, const float4v &v1) {
        *(uint4 *)p = make_uint4(pack_bf16x2(v0[0], v0[1]), pack_bf16x2(v0[2], v0[3]), pack_bf16x2(v1[0], v1[1]),
                                 pack_bf16x2(v1[2], v1[3]));
    };

    // first-layer features 8 q8 .. +7 of a fault from its inputs (x0, x1) = (tanh(L/8), lambda/8)
    // (the parameters are read from LDS at each use rather than held in registers)
    auto h0_group = [&](float x0, float x1) {
        const float4v *w0 = (const float4v *)(sv + SV_W0 + 16 * q8), *b0 = (const float4v *)(sv + SV_B0 + 8 * q8);
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; i++)
            v[i] = fmaxf(fmaf(w0[i >> 1][2 * (i & 1)], x0, fmaf(w0[i >> 1][2 * (i & 1) + 1], x1, b0[i >> 2][i & 3])), 0.f);
        return __builtin_bit_cast(bf16x8v, make_uint4(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]),
                                                      pack_bf16x2(v[4], v[5]), pack_bf16x2(v[6], v[7])));
    };
    // the slice's per-row inputs: x1 = lambda/8 once per launch, x0 = tanh(L/8) per shot
    float2 *X = (float2 *)(Cb + (size_t)(MP + 1) * 64);
    for (int r = t; r <= NP; r += blockDim.x) {
        const int j = r < NP ? A.perm[r] : -1;
        X[r] = make_float2(0.f, j >= 0 ? A.lam[j] * 0.125f : 0.f);
    }
    const uint32_t sentinel_off = (uint32_t)NP * 64u;

    const int total = A.list ? *A.list_count : A.count;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int shot = A.list ? A.list[item] : item;
        const uint8_t *syn = A.syn + (size_t)shot * m;
        const float *llr = A.llr + (size_t)shot * n;
        for (int i = t; i < m; i += blockDim.x) sg[i] = (syn[i] & 1) ? -1.f : 1.f;
        // the input layer is not stored: layer 0 recomputes a fault's first-layer features from
        // its 8-byte inputs wherever it needs them (padding rows get x0 = 0 and are never read)
        for (int r = t; r < NP; r += blockDim.x) {
            const int j = A.perm[r];
            X[r].x = j >= 0 ? tanhf(llr[j] * 0.125f) : 0.f;
        }
        __syncthreads();
        auto layer = [&](auto Lc) {
            constexpr int l = decltype(Lc)::value;
            // checks: c_i = relu((1/deg_i) sum_j A h_j + sigma_i a)
            {
                const bf16x8v a0 = frag(l * 3, 0), a1 = frag(l * 3, 1);
                const float4v av0 = *(const float4v *)(sv + SV_A + l * HID + 8 * q8);
                const float4v av1 = *(const float4v *)(sv + SV_A + l * HID + 8 * q8 + 4);
                for (int rt = wave; rt < MP / 16; rt += kBigWaves) {
                    const int i = rt * 16 + r16;
                    float4v acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
                    const uint32_t *nb = A.nbc + (size_t)i * dr;
                    uint32_t off[kGather];
#pragma unroll
                    for (int k = 0; k < kGather; k++) off[k] = k < dr ? nb[k] : sentinel_off;
                    for (int k0 = 0; k0 < dr; k0 += kGather) {
                        bf16x8v x[kGather];
                        if constexpr (l == 0) {
                            float2 xi[kGather];
#pragma unroll
                            for (int k = 0; k < kGather; k++) xi[k] = X[off[k] >> 6];
#pragma unroll
                            for (int k = 0; k < kGather; k++) {
                                // the zero row of padded lists stays zero
                                x[k] = off[k] == sentinel_off ? bf16x8v{} : h0_group(xi[k].x, xi[k].y);
                            }
                        } else {
#pragma unroll
                            for (int k = 0; k < kGather; k++) x[k] = gload(Hb, off[k] + q16);
                        }
#pragma unroll
                        for (int k = 0; k < kGather; k++)
                            off[k] = k0 + kGather + k < dr ? nb[k0 + kGather + k] : sentinel_off;
#pragma unroll
                        for (int k = 0; k < kGather; k++) {
                            acc0 = mfma32(a0, x[k], acc0);
                            acc1 = mfma32(a1, x[k], acc1);
                        }
                    }
                    const float rd = A.rdc[i], sgn = i < m ? sg[i] : 0.f;
                    float4v v0, v1;
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        v0[q] = fmaxf(rd * acc0[q] + sgn * av0[q], 0.f);
                        v1[q] = fmaxf(rd * acc1[q] + sgn * av1[q], 0.f);
                    }
                    store_group(Cb + (size_t)i * 64 + q16, v0, v1);
                }
            }
            __syncthreads();
            // faults: h_j = relu(B h_j + b + (1/deg_j) sum_i C c_i), b entering as the accumulator
            // of B h_j; in place (own rows only).  The last layer stores no features: it applies
            // the output layer to its bf16-rounded features and writes L' for its faults.
            {
                const bf16x8v b0 = frag(l * 3 + 1, 0), b1 = frag(l * 3 + 1, 1);
                const bf16x8v c0 = frag(l * 3 + 2, 0), c1 = frag(l * 3 + 2, 1);
                const float4v bv0 = *(const float4v *)(sv + SV_BL + l * HID + 8 * q8);
                const float4v bv1 = *(const float4v *)(sv + SV_BL + l * HID + 8 * q8 + 4);
                const int ntiles = NP / 16;
                // one pass: kFaultTiles tiles, each gathering D check rows per fault (the pass's
                // largest tile degree; the tables pad shorter lists with the zero row), every load
                // issued before the first product
                auto pass = [&](auto Dc, int rt0) {
                    constexpr int D = decltype(Dc)::value;
                    bf16x8v h[kFaultTiles], y[kFaultTiles][D];
                    float2 xo[kFaultTiles];
#pragma unroll
                    for (int tt = 0; tt < kFaultTiles; tt++) {
                        const int rt = rt0 + tt * kBigWaves;
                        const int r = (rt < ntiles ? rt : rt0) * 16 + r16;
                        if constexpr (l == 0) xo[tt] = X[r];
                        else h[tt] = gload(Hb, (uint32_t)r * 64u + q16);
                        const uint16_t *nb = nbf16 + (size_t)r * dc;
#pragma unroll
                        for (int k = 0; k < D; k++) y[tt][k] = gload(Cb, (uint32_t)nb[k] * 64u + q16);
                    }
#pragma unroll
                    for (int tt = 0; tt < kFaultTiles; tt++) {
                        const int rt = rt0 + tt * kBigWaves;
                        if (rt >= ntiles) continue;
                        const int r = rt * 16 + r16;
                        if constexpr (l == 0) h[tt] = h0_group(xo[tt].x, xo[tt].y);
                        float4v an0 = {0.f, 0.f, 0.f, 0.f}, an1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int k = 0; k < D; k++) {
                            an0 = mfma32(c0, y[tt][k], an0);
                            an1 = mfma32(c1, y[tt][k], an1);
                        }
                        if (D == kFaultGather) {  // tiles heavier than kFaultGather
                            const int dt = A.tdeg[rt];
                            for (int k = kFaultGather; k < dt; k++) {
                                const bf16x8v z = gload(Cb, (uint32_t)nbf16[(size_t)r * dc + k] * 64u + q16);
                                an0 = mfma32(c0, z, an0);
                                an1 = mfma32(c1, z, an1);
                            }
                        }
                        const float4v as0 = mfma32(b0, h[tt], bv0), as1 = mfma32(b1, h[tt], bv1);
                        const float rd = A.rdf[r];
                        float4v v0, v1;
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            v0[q] = fmaxf(rd * an0[q] + as0[q], 0.f);
                            v1[q] = fmaxf(rd * an1[q] + as1[q], 0.f);
                        }
                        if constexpr (l + 1 < NL) {
                            store_group(Hb + (size_t)r * 64 + q16, v0, v1);
                        } else {
                            // output layer: d_j = b_o + w . h_j over the bf16-rounded features,
                            // 8 per lane, then summed over the 4 lanes of the fault
                            const uint32_t w[4] = {pack_bf16x2(v0[0], v0[1]), pack_bf16x2(v0[2], v0[3]),
                                                   pack_bf16x2(v1[0], v1[1]), pack_bf16x2(v1[2], v1[3])};
                            const float4v *wo = (const float4v *)(sv + SV_W + 8 * q8);
                            float d = 0.f;
#pragma unroll
                            for (int i = 0; i < 4; i++) {
                                d += wo[i >> 1][2 * (i & 1)] * __uint_as_float(w[i] << 16);
                                d += wo[i >> 1][2 * (i & 1) + 1] * __uint_as_float(w[i] & 0xffff0000u);
                            }
                            d += __shfl_xor(d, 16, 64);
                            d += __shfl_xor(d, 32, 64);
                            const int j = A.perm[r];
                            if (q8 == 0 && j >= 0) A.llr_out[(size_t)shot * n + j] = llr[j] + (sv[SV_BO] + d);
                        }
                    }
                };
                for (int rt0 = wave; rt0 < ntiles; rt0 += kFaultTiles * kBigWaves) {
                    int D = 1;
#pragma unroll
                    for (int tt = 0; tt < kFaultTiles; tt++)
                        if (rt0 + tt * kBigWaves < ntiles) D = max(D, A.tdeg[rt0 + tt * kBigWaves]);
                    switch (D) {
                        case 1: pass(std::integral_constant<int, 1>{}, rt0); break;
                        case 2: pass(std::integral_constant<int, 2>{}, rt0); break;
                        case 3: pass(std::integral_constant<int, 3>{}, rt0); break;
                        case 4: pass(std::integral_constant<int, 4>{}, rt0); break;
                        case 5: pass(std::integral_constant<int, 5>{}, rt0); break;
                        default: pass(std::integral_constant<int, kFaultGather>{}, rt0); break;
                    }
                }
            }
            __syncthreads();
        };
        static_assert(NL == 3, "layers are instantiated one by one");
        layer(std::integral_constant<int, 0>{});
        layer(std::integral_constant<int, 1>{});
        layer(std::integral_constant<int, 2>{});
    }
}

__global__ void zero_f32(float *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

__global__ void adam_kernel(float *theta, const float *grad, float *m1, float *m2, int n, float lr, float b1t, float b2t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float a = 0.9f * m1[i] + 0.1f * g;
    const float b = 0.999f * m2[i] + 0.001f * g * g;
    m1[i] = a;
    m2[i] = b;
    theta[i] -= lr * (a / (1.f - b1t)) / (sqrtf(b / (1.f - b2t)) + 1e-8f);
}

}  // namespace

static size_t net_shared_bytes(const DevGraph &g, bool train) {
    size_t o[5];
    return net_shared_layout(g.n, g.m, g.nnz, train, o);
}
static size_t net_act_bytes(const DevGraph &g, bool train) {
    size_t o[5];
    return net_act_layout(g.n, g.m, train, o);
}
size_t net_lds_bytes(const DevGraph &g, bool train) { return net_shared_bytes(g, train) + net_act_bytes(g, train); }

// Wavefronts per inference workgroup: 11 in one workgroup when they fit in a CU's 160 KB of LDS
// (11 wavefronts need 170 VGPRs or fewer: three per SIMD), else 5 (two workgroups per CU).
static int infer_waves(const DevGraph &g) {
    const size_t sh = infer_shared_bytes(g.n, g.m, g.max_rw, g.max_cw), w = infer_wave_bytes(g.n, g.m, infer_regular(g));
    return sh + (size_t)kInferWavesMax * w <= 160 * 1024 ? kInferWavesMax : 5;
}
static size_t infer_lds_bytes(const DevGraph &g) {
    return infer_shared_bytes(g.n, g.m, g.max_rw, g.max_cw) +
           (size_t)infer_waves(g) * infer_wave_bytes(g.n, g.m, infer_regular(g));
}

// Inference launch: grid sized for the device, one wavefront per shot; the neighbour loops are
// unrolled for codes of maximum row / column weight 6 / 3 (the bivariate bicycle codes), and run
// to the code's maximum weights otherwise.
template <int UR, int UF>
static hipError_t launch_infer_t(const NetArgs &a, int max_items, int num_cus, hipStream_t st) {
    const size_t lds = infer_lds_bytes(a.g);
    hipError_t e = hipFuncSetAttribute((const void *)net_infer_kernel<UR, UF>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int nw = infer_waves(a.g);
    const int per_cu = std::max<int>(1, (int)((160 * 1024) / lds));
    const int grid = std::max(1, std::min((max_items + nw - 1) / nw, num_cus * per_cu));
    hipLaunchKernelGGL((net_infer_kernel<UR, UF>), dim3(grid), dim3(64 * nw), lds, st, a);
    return hipGetLastError();
}
static hipError_t launch_infer(const NetArgs &a, int max_items, int num_cus, hipStream_t st) {
    if (a.g.max_rw == 6 && a.g.max_cw == 3) return launch_infer_t<6, 3>(a, max_items, num_cus, st);
    return launch_infer_t<0, 0>(a, max_items, num_cus, st);
}

}  // namespace qlsd

using namespace qlsd;

struct qlsd_net_s {
    qlsd_code code;
    DevGraph g;
    float *d_lam = nullptr, *d_theta = nullptr, *d_m1 = nullptr, *d_m2 = nullptr, *d_grad = nullptr, *d_loss = nullptr;
    int step = 0;
    int num_cus = 0;
    bool wave_infer = false;          // inference by net_infer_kernel (LDS-resident, wave per shot)
    unsigned char *d_act = nullptr;   // training activations when they do not fit in LDS (lazy)
    size_t act_stride = 0;
    int act_slices = 0;
    // large-graph inference (net_infer_big_kernel): neighbour tables, and the net's own feature
    // workspace for qlsd_net_forward (decoders bring their own, see qlsd_decoder_set_net)
    uint32_t *d_nbc = nullptr, *d_nbf = nullptr;
    float *d_rdc = nullptr, *d_rdf = nullptr;
    int32_t *d_perm = nullptr, *d_rowof = nullptr, *d_tdeg = nullptr;  // fault rows sorted by degree
    unsigned char *d_iws = nullptr;
};

namespace qlsd {
// Training, gradient and (for graphs the wave kernel cannot hold) inference launch of net_kernel:
// one workgroup per shot at a time; activations in LDS or in the net's workspace slices.
static hipError_t launch_net(qlsd_net_s *net, NetArgs a, int grid, hipStream_t st) {
    const bool train = a.train != 0;
    size_t lds = net_shared_bytes(a.g, train);
    if (net->act_stride && !net->d_act &&
        hipMalloc((void **)&net->d_act, net->act_stride * net->act_slices) != hipSuccess) {
        net->d_act = nullptr;
        return hipErrorOutOfMemory;
    }
    if (net->d_act) {
        a.act = net->d_act;
        a.act_stride = net->act_stride;
        grid = std::min(grid, net->act_slices);
    } else {
        lds += net_act_bytes(a.g, train);
    }
    hipError_t e = hipFuncSetAttribute((const void *)net_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(net_kernel, dim3(std::max(grid, 1)), dim3(kNetThreads), lds, st, a);
    return hipGetLastError();
}
// Slices of the large-graph inference workspace: one per compute unit, so the grid's features
// (about 0.7 MB per slice for the detector error model) stay in the last-level cache.
static int big_slices(const qlsd_net_s *net) { return net->num_cus; }
size_t net_infer_workspace_bytes(const qlsd_net_s *net) {
    return net->wave_infer ? 0 : big_slice_bytes(net->g.n, net->g.m) * (size_t)big_slices(net);
}
static hipError_t launch_infer_big(const qlsd_net_s *net, NetArgs a, unsigned char *ws, int max_items, hipStream_t st) {
    a.act = ws;
    a.act_stride = big_slice_bytes(a.g.n, a.g.m);
    a.nbc = net->d_nbc;
    a.nbf = net->d_nbf;
    a.rdc = net->d_rdc;
    a.rdf = net->d_rdf;
    a.perm = net->d_perm;
    a.tdeg = net->d_tdeg;
    const int grid = std::max(1, std::min(max_items, big_slices(net)));
    const size_t lds = big_dyn_lds(a.g);
    hipError_t e = hipFuncSetAttribute((const void *)net_infer_big_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(net_infer_big_kernel, dim3(grid), dim3(64 * kBigWaves), lds, st, a);
    return hipGetLastError();
}
// Inference of max_items shots (a.list / a.count say which); ws: a feature workspace of
// net_infer_workspace_bytes(net) for large graphs (nullptr: the net's own).
static hipError_t run_forward(qlsd_net_s *net, const NetArgs &a, int max_items, unsigned char *ws, hipStream_t st) {
    if (net->wave_infer) return launch_infer(a, max_items, net->num_cus, st);
    if (!ws) {
        if (!net->d_iws && hipMalloc((void **)&net->d_iws, net_infer_workspace_bytes(net)) != hipSuccess) {
            net->d_iws = nullptr;
            return hipErrorOutOfMemory;
        }
        ws = net->d_iws;
    }
    return launch_infer_big(net, a, ws, max_items, st);
}
}  // namespace qlsd

extern "C" {

qlsd_status qlsd_net_create(qlsd_code code, const double *priors, const float *params, qlsd_net *out) {
    if (!out || !code || !priors || !params) { set_last_error("NULL argument"); return QLSD_E_INVALID; }
    *out = nullptr;
    const DevGraph g = code_graph(code);
    // u16 CSR/CSC tables in LDS next to the weights
    if (g.n >= 65535 || g.nnz >= 65535 || net_shared_bytes(g, true) > 159 * 1024) {
        set_last_error("graph too large for the refinement network (u16 tables in LDS)");
        return QLSD_E_UNSUPPORTED;
    }
    std::vector<float> lam(g.n);
    for (int j = 0; j < g.n; j++) {
        if (!(priors[j] > 0.0 && priors[j] < 1.0)) { set_last_error("prior %d not in (0,1)", j); return QLSD_E_PRIOR; }
        lam[j] = (float)log((1.0 - priors[j]) / priors[j]);
    }
    qlsd_net net = new (std::nothrow) qlsd_net_s();
    if (!net) { set_last_error("host allocation failed"); return QLSD_E_NOMEM; }
    net->code = code;
    net->g = g;
    bool ok = hipMalloc((void **)&net->d_lam, sizeof(float) * g.n) == hipSuccess &&
              hipMalloc((void **)&net->d_theta, sizeof(float) * NPAR) == hipSuccess &&
              hipMalloc((void **)&net->d_m1, sizeof(float) * NPAR) == hipSuccess &&
              hipMalloc((void **)&net->d_m2, sizeof(float) * NPAR) == hipSuccess &&
              hipMalloc((void **)&net->d_grad, sizeof(float) * NPAR) == hipSuccess &&
              hipMalloc((void **)&net->d_loss, sizeof(float) * 4) == hipSuccess &&
              hipMemcpy(net->d_lam, lam.data(), sizeof(float) * g.n, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(net->d_theta, params, sizeof(float) * NPAR, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemset(net->d_m1, 0, sizeof(float) * NPAR) == hipSuccess &&
              hipMemset(net->d_m2, 0, sizeof(float) * NPAR) == hipSuccess;
    int dev = 0;
    hipDeviceProp_t prop;
    ok = ok && hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess;
    if (!ok) {
        qlsd_net_destroy(net);
        set_last_error("device allocation failed");
        return QLSD_E_NOMEM;
    }
    net->num_cus = prop.multiProcessorCount;
    // wave-per-shot inference needs u16 byte offsets of feature rows (64 B each) and LDS room
    net->wave_infer = pad16(g.n) + 1 <= 1023 && pad16(g.m) + 1 <= 1023 && infer_lds_bytes(g) <= 160 * 1024;
    if (net_lds_bytes(g, true) > 159 * 1024) {  // training activations in a device workspace (allocated at first use)
        net->act_stride = (net_act_bytes(g, true) + 255) & ~size_t(255);
        net->act_slices = net->num_cus;
    }
    if (!net->wave_infer) {
        const int NP = pad16(g.n), MP = pad16(g.m);
        if (MP + 1 > 65535 || big_dyn_lds(g) + 20 * 1024 > 159 * 1024) {
            qlsd_net_destroy(net);
            set_last_error("graph too large for the refinement's inference kernel");
            return QLSD_E_UNSUPPORTED;
        }
        std::vector<int32_t> col_ptr(g.n + 1), perm, rowof, tdeg;
        ok = (size_t)(NP + 1) * 64 < (1ull << 32) && (size_t)(MP + 1) * 64 < (1ull << 32) &&
             hipMemcpy(col_ptr.data(), g.col_ptr, sizeof(int32_t) * (g.n + 1), hipMemcpyDeviceToHost) == hipSuccess;
        if (ok) big_fault_order(col_ptr, g.n, perm, rowof, tdeg);
        ok = ok && hipMalloc((void **)&net->d_nbc, sizeof(uint32_t) * (size_t)MP * g.max_rw) == hipSuccess &&
             hipMalloc((void **)&net->d_nbf, sizeof(uint32_t) * (size_t)NP * g.max_cw) == hipSuccess &&
             hipMalloc((void **)&net->d_rdc, sizeof(float) * MP) == hipSuccess &&
             hipMalloc((void **)&net->d_rdf, sizeof(float) * NP) == hipSuccess &&
             hipMalloc((void **)&net->d_perm, sizeof(int32_t) * NP) == hipSuccess &&
             hipMalloc((void **)&net->d_rowof, sizeof(int32_t) * g.n) == hipSuccess &&
             hipMalloc((void **)&net->d_tdeg, sizeof(int32_t) * (NP / 16)) == hipSuccess &&
             hipMemcpy(net->d_perm, perm.data(), sizeof(int32_t) * NP, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(net->d_rowof, rowof.data(), sizeof(int32_t) * g.n, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(net->d_tdeg, tdeg.data(), sizeof(int32_t) * (NP / 16), hipMemcpyHostToDevice) == hipSuccess;
        if (ok) {
            hipLaunchKernelGGL(big_tables_kernel, dim3(256), dim3(256), 0, 0, g, net->d_perm, net->d_rowof, net->d_nbc,
                               net->d_nbf, net->d_rdc, net->d_rdf);
            ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
        }
        if (!ok) {
            qlsd_net_destroy(net);
            set_last_error("device allocation of the inference tables failed");
            return QLSD_E_NOMEM;
        }
    }
    *out = net;
    return QLSD_OK;
}

qlsd_status qlsd_net_set_priors(qlsd_net net, const double *priors) {
    if (!net || !priors) { set_last_error("NULL argument"); return QLSD_E_INVALID; }
    std::vector<float> lam(net->g.n);
    for (int j = 0; j < net->g.n; j++) {
        if (!(priors[j] > 0.0 && priors[j] < 1.0)) { set_last_error("prior %d not in (0,1)", j); return QLSD_E_PRIOR; }
        lam[j] = (float)log((1.0 - priors[j]) / priors[j]);
    }
    if (hipMemcpy(net->d_lam, lam.data(), sizeof(float) * net->g.n, hipMemcpyHostToDevice) != hipSuccess) {
        set_last_error("hipMemcpy failed");
        return QLSD_E_DEVICE;
    }
    return QLSD_OK;
}

qlsd_status qlsd_net_set_params(qlsd_net net, const float *params) {
    if (!net || !params) { set_last_error("NULL argument"); return QLSD_E_INVALID; }
    if (hipMemcpy(net->d_theta, params, sizeof(float) * NPAR, hipMemcpyHostToDevice) != hipSuccess) {
        set_last_error("hipMemcpy failed");
        return QLSD_E_DEVICE;
    }
    return QLSD_OK;
}

qlsd_status qlsd_net_get_params(qlsd_net net, float *params) {
    if (!net || !params) { set_last_error("NULL argument"); return QLSD_E_INVALID; }
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(params, net->d_theta, sizeof(float) * NPAR, hipMemcpyDeviceToHost) != hipSuccess) {
        set_last_error("hipMemcpy failed");
        return QLSD_E_DEVICE;
    }
    return QLSD_OK;
}

static NetArgs net_args(qlsd_net net) {
    NetArgs a;
    memset(&a, 0, sizeof(a));
    a.g = net->g;
    a.lam = net->d_lam;
    a.theta = net->d_theta;
    return a;
}

qlsd_status qlsd_net_forward(qlsd_net net, const uint8_t *syndromes, const float *llr, int32_t B, float *llr_out,
                             void *stream) {
    if (!net || B < 0 || (B > 0 && (!syndromes || !llr || !llr_out))) { set_last_error("bad arguments"); return QLSD_E_INVALID; }
    if (B == 0) return QLSD_OK;
    NetArgs a = net_args(net);
    a.syn = syndromes;
    a.llr = llr;
    a.llr_out = llr_out;
    a.count = B;
    if (run_forward(net, a, B, nullptr, (hipStream_t)stream) != hipSuccess) {
        set_last_error("net launch failed");
        return QLSD_E_DEVICE;
    }
    return QLSD_OK;
}

static qlsd_status grad_impl(qlsd_net net, const uint8_t *syn, const float *llr, const uint8_t *err, int32_t B,
                             float *grad, float *loss, hipStream_t st) {
    hipLaunchKernelGGL(zero_f32, dim3((NPAR + 255) / 256), dim3(256), 0, st, grad, NPAR);
    hipLaunchKernelGGL(zero_f32, dim3(1), dim3(64), 0, st, loss, 1);
    NetArgs a = net_args(net);
    a.syn = syn;
    a.llr = llr;
    a.err = err;
    a.count = B;
    a.grad = grad;
    a.loss = loss;
    a.inv_total = 1.f / ((float)B * (float)net->g.n);
    a.train = 1;
    const int grid = std::min(B, net->num_cus);
    if (launch_net(net, a, grid, st) != hipSuccess) { set_last_error("net launch failed"); return QLSD_E_DEVICE; }
    return QLSD_OK;
}

qlsd_status qlsd_net_gradient(qlsd_net net, const uint8_t *syndromes, const float *llr, const uint8_t *errors,
                              int32_t B, float *grad, float *loss, void *stream) {
    if (!net || B < 1 || !syndromes || !llr || !errors || !grad || !loss) { set_last_error("bad arguments"); return QLSD_E_INVALID; }
    return grad_impl(net, syndromes, llr, errors, B, grad, loss, (hipStream_t)stream);
}

qlsd_status qlsd_net_train_step(qlsd_net net, const uint8_t *syndromes, const float *llr, const uint8_t *errors,
                                int32_t B, float lr, void *stream) {
    if (!net || B < 1 || !syndromes || !llr || !errors) { set_last_error("bad arguments"); return QLSD_E_INVALID; }
    hipStream_t st = (hipStream_t)stream;
    qlsd_status s = grad_impl(net, syndromes, llr, errors, B, net->d_grad, net->d_loss, st);
    if (s != QLSD_OK) return s;
    net->step++;
    const float b1t = powf(0.9f, (float)net->step), b2t = powf(0.999f, (float)net->step);
    hipLaunchKernelGGL(adam_kernel, dim3((NPAR + 255) / 256), dim3(256), 0, st, net->d_theta, net->d_grad, net->d_m1,
                       net->d_m2, NPAR, lr, b1t, b2t);
    if (hipGetLastError() != hipSuccess) { set_last_error("adam launch failed"); return QLSD_E_DEVICE; }
    return QLSD_OK;
}

void qlsd_net_destroy(qlsd_net net) {
    if (!net) return;
    hipFree(net->d_lam);
    hipFree(net->d_theta);
    hipFree(net->d_m1);
    hipFree(net->d_m2);
    hipFree(net->d_grad);
    hipFree(net->d_loss);
    hipFree(net->d_act);
    hipFree(net->d_nbc);
    hipFree(net->d_nbf);
    hipFree(net->d_rdc);
    hipFree(net->d_rdf);
    hipFree(net->d_perm);
    hipFree(net->d_rowof);
    hipFree(net->d_tdeg);
    hipFree(net->d_iws);
    delete net;
}

}  // extern "C"

namespace qlsd {
// Refinement of the LLRs of the listed shots, in place (decode path).
hipError_t net_refine_listed(qlsd_net_s *net, const float *lam, const uint8_t *syn, float *llr, const int *list,
                             const int *list_count, int max_count, unsigned char *ws, hipStream_t st) {
    NetArgs a = net_args(net);
    a.lam = lam;  // the decoder's prior LLRs, so one net serves decoders of any noise strength
    a.syn = syn;
    a.llr = llr;
    a.llr_out = llr;
    a.list = list;
    a.list_count = list_count;
    a.count = max_count;
    return run_forward(net, a, max_count, ws, st);
}
void net_graph_dims(const qlsd_net_s *net, int *m, int *n) {
    *m = net->g.m;
    *n = net->g.n;
}
const float *net_loss_ptr(qlsd_net net) { return net->d_loss; }
}  // namespace qlsd
