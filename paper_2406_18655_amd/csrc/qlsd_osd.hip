// Global OSD-0 post-processing on the GPU: the comparator LSD is measured against.
//
// What is computed (Hillmann et al., Sec. 2.2, inversion decoding; the reliability order of
// Sec. 4.1 step 2): all n columns of H in ascending key (llr_j, j) -- the faults most likely in
// error first -- are reduced one after another into a single Gauss-Jordan basis over all m
// detectors; a column is a pivot iff it is independent of the columns before it, and e_hat is
// the unique solution of H e = s supported on the pivot columns.  Greedy pivot sets are
// prefix-consistent and the solution on a pivot set is unique, so the reduction stops as soon as
// the syndrome lies in the span of the pivots found so far (the later pivots would carry zeros);
// a syndrome outside the image of H runs through every column and is flagged UNSAT with a zero
// correction.
//
// MI355X mapping: one wavefront per shot.  The shot's keys are sorted in LDS by a bitonic
// network of wave-wide compare-exchange passes; the basis is the bit-sliced one of the LSD
// kernels (lane l holds detector rows l, l + 64, ...), in registers for m <= 256 and in the
// workgroup's slice of device memory for m <= 1024.
#include "qlsd_lsd_dev.h"

namespace qlsd {

namespace {

template <int W, bool WIDE>
__device__ void osd0_shot(const OsdArgs &A, uint64_t *keys, uint32_t *cbit, int32_t *colAt, int shot, int lane,
                          uint64_t *basis_mem) {
    const int m = A.g.m, n = A.g.n, P = A.P;
    const float *llr = A.llr + (size_t)shot * n;
    const uint8_t *syn = A.syn + (size_t)shot * m;
    uint8_t *corr = A.corr + (size_t)shot * n;
    bool nan = false;
    for (int j = lane; j < P; j += 64) {
        uint64_t key = ~0ull;  // padding sorts last
        if (j < n) {
            const float v = llr[j];
            nan |= (v != v);
            key = ((uint64_t)ordered_key(v) << 32) | (uint32_t)j;
        }
        keys[j] = key;
    }
    for (int w = lane; w < (n + 31) / 32; w += 64) cbit[w] = 0u;
    uint64_t sp0[W];
#pragma unroll
    for (int s = 0; s < W; s++) {
        const int r = s * 64 + lane;
        sp0[s] = ballot(r < m && (syn[r < m ? r : 0] & 1));
    }
    wave_sync();
    auto finish = [&](uint8_t st, int cols) {
        wave_sync();
        for (int j = lane; j < n; j += 64) corr[j] = (uint8_t)((cbit[j >> 5] >> (j & 31)) & 1u);
        if (A.info && lane == 0) {
            qlsd_shot_info inf;
            inf.status = st;
            inf.reserved = 0;
            inf.bp_iters = (int16_t)A.bp_iters;
            inf.n_clusters = 1;
            inf.rounds = (int16_t)(cols < 32767 ? cols : 32767);
            inf.max_cluster_cols = cols;
            A.info[shot] = inf;
        }
    };
    if (ballot(nan)) { finish(QLSD_ST_LSD_RUN | QLSD_ST_BAD_LLR, 0); return; }

    // ascending bitonic sort of the P keys
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < P; i += 64) {
                const int l = i ^ j;
                if (l > i) {
                    const uint64_t a = keys[i], b = keys[l];
                    if ((a > b) == ((i & k) == 0)) { keys[i] = b; keys[l] = a; }
                }
            }
            wave_sync();
        }
    }

    Basis<W, WIDE> B;
    if constexpr (WIDE) {
        B.mem = basis_mem + lane;
        const int msl = (m + 63) >> 6;
        for (int s = 0; s < msl; s++)
            for (int w = 0; w < msl; w++) { B.M(s, w) = 0; B.C(s, w) = 0; }
        B.ns = msl;
    } else {
        B.ns = W;
    }
    bool any = false;
#pragma unroll
    for (int s = 0; s < W; s++) {
        if constexpr (!WIDE) {
#pragma unroll
            for (int w = 0; w < W; w++) { B.M(s, w) = 0; B.C(s, w) = 0; }
        }
        B.piv[s] = 0;
        B.sp[s] = sp0[s];
        any |= sp0[s] != 0;
    }
    if (!any) { finish(QLSD_ST_LSD_RUN, 0); return; }
    LsdLds S;
    S.colAt = colAt;
    wave_sync();
    int t = 0;
    bool spanned = false;
    while (t < n && !spanned) {
        const int col = __builtin_amdgcn_readfirstlane((int)(uint32_t)keys[t]);
        const int c0 = __builtin_amdgcn_readfirstlane(A.g.col_ptr[col]);
        const int cw = __builtin_amdgcn_readfirstlane(A.g.col_ptr[col + 1]) - c0;
        const int lr = lane < cw ? A.g.row_idx[c0 + lane] : -1;
        insert_column<W>(B, S, col, lane, lr, 0, cw);
        t++;
        uint64_t rest = 0;
#pragma unroll
        for (int s = 0; s < W; s++) rest |= B.sp[s];
        spanned = rest == 0;
    }
    if (!spanned) { finish(QLSD_ST_LSD_RUN | QLSD_ST_UNSAT, t); return; }
    wave_sync();
    // solution on the pivot columns: a pivot row's column is set iff its combination of the
    // syndrome's pivot rows has odd parity
    uint64_t as[W];
#pragma unroll
    for (int s = 0; s < W; s++) as[s] = sp0[s] & B.piv[s];
#pragma unroll
    for (int s = 0; s < W; s++) {
        const bool set = ((B.piv[s] >> lane) & 1ull) && parity_C<W>(B, s, as);
        if (set) {
            const int col = colAt[s * 64 + lane];
            atomicOr(&cbit[col >> 5], 1u << (col & 31));
        }
    }
    finish(QLSD_ST_LSD_RUN, t);
}

template <int W, bool WIDE>
__global__ __launch_bounds__(WIDE ? 64 : 256) void osd0_kernel(OsdArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned char *base = smem + (size_t)wid * A.wave_bytes;
    uint64_t *keys = (uint64_t *)base;
    int32_t *colAt = (int32_t *)(keys + A.P);
    uint32_t *cbit = (uint32_t *)(colAt + 64 * W);
    uint64_t *mem = WIDE ? A.ws + (size_t)blockIdx.x * (2 * W * W * 64) : nullptr;
    const int total = A.list ? *A.list_count : A.count;
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(A.next_item, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= total) break;
        osd0_shot<W, WIDE>(A, keys, cbit, colAt, A.list ? A.list[item] : item, lane, mem);
        wave_sync();
    }
}

}  // namespace

size_t osd0_wave_bytes(const DevGraph &g, int W, int P) {
    return ((size_t)P * 8 + (size_t)64 * W * 4 + (size_t)((g.n + 31) / 32) * 4 + 15) & ~(size_t)15;
}

hipError_t launch_osd0(const OsdArgs &a, int W, int grid, hipStream_t st) {
    const int waves = W == kWideW ? 1 : kLsdThreads / 64;
    const size_t lds = (size_t)a.wave_bytes * waves;
    const void *fn = nullptr;
    switch (W) {
        case 1: fn = (const void *)osd0_kernel<1, false>; break;
        case 2: fn = (const void *)osd0_kernel<2, false>; break;
        case 4: fn = (const void *)osd0_kernel<4, false>; break;
        case kWideW: fn = (const void *)osd0_kernel<kWideW, true>; break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    switch (W) {
        case 1: hipLaunchKernelGGL((osd0_kernel<1, false>), dim3(grid), dim3(256), lds, st, a); break;
        case 2: hipLaunchKernelGGL((osd0_kernel<2, false>), dim3(grid), dim3(256), lds, st, a); break;
        case 4: hipLaunchKernelGGL((osd0_kernel<4, false>), dim3(grid), dim3(256), lds, st, a); break;
        default: hipLaunchKernelGGL((osd0_kernel<kWideW, true>), dim3(grid), dim3(64), lds, st, a); break;
    }
    return hipGetLastError();
}

}  // namespace qlsd
