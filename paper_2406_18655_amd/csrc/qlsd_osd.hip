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
// Global OSD-CS of order w (the comparator at higher order; m <= 256): the same elimination run
// through every column, which lists the dependent (non-pivot) columns T in key order, then the
// combination sweep LSD-mu applies per cluster applied to the whole matrix -- the OSD-0
// solution, every single column of T, every pair among the first min(w, |T|) -- each scored by
// the integer weight of its solution; the strictly smallest weight wins, ties to the candidate
// met first.  A column t of T changes the pivot part by z_t, the pivot columns whose combination
// equals column t, read off the final basis.
//
// MI355X mapping: one wavefront per shot.  The shot's keys are sorted in LDS by a bitonic
// network of wave-wide compare-exchange passes; the basis is the bit-sliced one of the LSD
// kernels (lane l holds detector rows l, l + 64, ...), in registers for m <= 256 and in the
// workgroup's slice of device memory for m <= 1024.
#include "qlsd_lsd_dev.h"

namespace qlsd {

namespace {

// z: the pivot columns whose combination reproduces column col, as pivot rows (global basis:
// local rows are detectors).
template <int W, class BB>
__device__ __forceinline__ void global_column_combination(const DevGraph &g, const BB &B, int col, int lane,
                                                          uint64_t (&z)[W]) {
    uint32_t bf = 0;
    for (int e = g.col_ptr[col]; e < g.col_ptr[col + 1]; e++) {
        const int r = g.row_idx[e];
        if ((r & 63) == lane) bf |= 1u << (r >> 6);
    }
    uint64_t a[W];
#pragma unroll
    for (int s = 0; s < W; s++) a[s] = ballot((bf >> s) & 1u) & B.piv[s];
#pragma unroll
    for (int s = 0; s < W; s++) z[s] = ballot(((B.piv[s] >> lane) & 1ull) && parity_C<W>(B, s, a));
}

template <int W, bool WIDE, bool CS>
__device__ void osd0_shot(const OsdArgs &A, uint64_t *keys, uint32_t *cbit, int32_t *colAt, const OsdCsLds &X,
                          int shot, int lane, uint64_t *basis_mem) {
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
    // a zero syndrome: OSD-0's answer is zero; OSD-CS still sweeps (a column of negative weight,
    // a prior above 1/2, could make a nonzero solution lighter)
    if (!any && !CS) { finish(QLSD_ST_LSD_RUN, 0); return; }
    LsdLds S;
    S.colAt = colAt;
    S.wq = X.wq;
    wave_sync();
    int t = 0, nd = 0;
    bool spanned = false;
    // OSD-0 stops once the syndrome is in the span (later pivots would carry zeros); OSD-CS
    // needs every dependent column, so it runs through all of them
    while (t < n && (CS || !spanned)) {
        const int col = __builtin_amdgcn_readfirstlane((int)(uint32_t)keys[t]);
        const int c0 = __builtin_amdgcn_readfirstlane(A.g.col_ptr[col]);
        const int cw = __builtin_amdgcn_readfirstlane(A.g.col_ptr[col + 1]) - c0;
        const int lr = lane < cw ? A.g.row_idx[c0 + lane] : -1;
        const bool piv = insert_column<W>(B, S, col, lane, lr, 0, cw);
        if constexpr (CS) {
            if (!piv) {
                if (lane == 0) X.dep[nd] = col;
                nd++;
            }
        }
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
    uint64_t as[W], x[W];
#pragma unroll
    for (int s = 0; s < W; s++) as[s] = sp0[s] & B.piv[s];
#pragma unroll
    for (int s = 0; s < W; s++) x[s] = ballot(((B.piv[s] >> lane) & 1ull) && parity_C<W>(B, s, as));
    if constexpr (CS) {
        // combination sweep over T (dep[0 .. nd), ascending key)
#pragma unroll
        for (int s = 0; s < W; s++)
            if ((B.piv[s] >> lane) & 1ull) X.wq[s * 64 + lane] = A.omega[colAt[s * 64 + lane]];
        const int w = A.cs_order < nd ? A.cs_order : nd;
        for (int a = 0; a < w; a++) {
            const int col = __builtin_amdgcn_readfirstlane(X.dep[a]);
            uint64_t z[W];
            global_column_combination<W>(A.g, B, col, lane, z);
            if (lane == 0) {
#pragma unroll
                for (int s = 0; s < W; s++) X.zk[a * W + s] = z[s];
                X.tw[a] = A.omega[col];
            }
        }
        wave_sync();
        const int64_t cost0 = pivot_cost<W>(S, x);
        // singles: every column of T; the first of equal cost wins
        int64_t bs_cost = INT64_MAX;
        int bs = -1;
        for (int e = 0; e < nd; e++) {
            const int col = __builtin_amdgcn_readfirstlane(X.dep[e]);
            uint64_t z[W], y[W];
            global_column_combination<W>(A.g, B, col, lane, z);
#pragma unroll
            for (int s = 0; s < W; s++) y[s] = x[s] ^ z[s];
            const int64_t cost = pivot_cost<W>(S, y) + A.omega[col];
            if (cost < bs_cost) { bs_cost = cost; bs = e; }
        }
        // pairs (a, b), a < b < w, lexicographic; spread over the lanes, the smallest
        // (cost, pair index) kept
        const int npair = w * (w - 1) / 2;
        uint64_t bp = ~0ull;
        for (int p = lane; p < npair; p += 64) {
            int a = 0, rem = p;
            while (rem >= w - 1 - a) { rem -= w - 1 - a; a++; }
            const int b = a + 1 + rem;
            uint64_t y[W];
#pragma unroll
            for (int s = 0; s < W; s++) y[s] = x[s] ^ X.zk[a * W + s] ^ X.zk[b * W + s];
            const int64_t cost = pivot_cost<W>(S, y) + X.tw[a] + X.tw[b];
            const uint64_t key = ((uint64_t)(cost + (1ll << 50)) << 12) | (uint64_t)p;
            bp = key < bp ? key : bp;
        }
        bp = wave_min_u64(bp);
        const int64_t bp_cost = bp == ~0ull ? INT64_MAX : (int64_t)(bp >> 12) - (1ll << 50);
        if (bs_cost < cost0 && bs_cost <= bp_cost) {
            const int col = __builtin_amdgcn_readfirstlane(X.dep[bs]);
            uint64_t z[W];
            global_column_combination<W>(A.g, B, col, lane, z);
#pragma unroll
            for (int s = 0; s < W; s++) x[s] ^= z[s];
            if (lane == 0) atomicOr(&cbit[col >> 5], 1u << (col & 31));
        } else if (bp_cost < cost0 && bp_cost < bs_cost) {
            const int p = (int)(bp & 4095ull);
            int a = 0, rem = p;
            while (rem >= w - 1 - a) { rem -= w - 1 - a; a++; }
            const int b = a + 1 + rem;
#pragma unroll
            for (int s = 0; s < W; s++) x[s] ^= X.zk[a * W + s] ^ X.zk[b * W + s];
            if (lane == 0) {
                const int ca = X.dep[a], cb = X.dep[b];
                atomicOr(&cbit[ca >> 5], 1u << (ca & 31));
                atomicOr(&cbit[cb >> 5], 1u << (cb & 31));
            }
        }
    }
#pragma unroll
    for (int s = 0; s < W; s++) {
        if ((x[s] >> lane) & 1ull) {
            const int col = colAt[s * 64 + lane];
            atomicOr(&cbit[col >> 5], 1u << (col & 31));
        }
    }
    finish(QLSD_ST_LSD_RUN, t);
}

template <int W, bool WIDE, bool CS>
__global__ __launch_bounds__(WIDE ? 64 : 256) void osd0_kernel(OsdArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned char *base = smem + (size_t)wid * A.wave_bytes;
    uint64_t *keys = (uint64_t *)base;
    int32_t *colAt = (int32_t *)(keys + A.P);
    uint32_t *cbit = (uint32_t *)(colAt + 64 * W);
    OsdCsLds X;  // OSD-CS arrays after the OSD-0 block (8-byte aligned)
    {
        unsigned char *q = base + osd0_wave_bytes_w(A.g.n, W, A.P, false);
        X.wq = (int64_t *)q;
        X.zk = (uint64_t *)(X.wq + 64 * W);
        X.tw = (int64_t *)(X.zk + kOsdCsMaxOrder * W);
        X.dep = (int32_t *)(X.tw + kOsdCsMaxOrder);
    }
    uint64_t *mem = WIDE ? A.ws + (size_t)blockIdx.x * (2 * W * W * 64) : nullptr;
    const int total = A.list ? *A.list_count : A.count;
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(A.next_item, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= total) break;
        osd0_shot<W, WIDE, CS>(A, keys, cbit, colAt, X, A.list ? A.list[item] : item, lane, mem);
        wave_sync();
    }
}

}  // namespace

size_t osd0_wave_bytes(const DevGraph &g, int W, int P, bool cs) { return osd0_wave_bytes_w(g.n, W, P, cs); }

template <bool CS>
static hipError_t launch_osd_t(const OsdArgs &a, int W, int grid, hipStream_t st) {
    const int waves = W == kWideW ? 1 : kLsdThreads / 64;
    const size_t lds = (size_t)a.wave_bytes * waves;
    const void *fn = nullptr;
    switch (W) {
        case 1: fn = (const void *)osd0_kernel<1, false, CS>; break;
        case 2: fn = (const void *)osd0_kernel<2, false, CS>; break;
        case 4: fn = (const void *)osd0_kernel<4, false, CS>; break;
        case kWideW:
            if (CS) return hipErrorInvalidValue;
            fn = (const void *)osd0_kernel<kWideW, true, false>;
            break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    switch (W) {
        case 1: hipLaunchKernelGGL((osd0_kernel<1, false, CS>), dim3(grid), dim3(256), lds, st, a); break;
        case 2: hipLaunchKernelGGL((osd0_kernel<2, false, CS>), dim3(grid), dim3(256), lds, st, a); break;
        case 4: hipLaunchKernelGGL((osd0_kernel<4, false, CS>), dim3(grid), dim3(256), lds, st, a); break;
        default: hipLaunchKernelGGL((osd0_kernel<kWideW, true, false>), dim3(grid), dim3(64), lds, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_osd0(const OsdArgs &a, int W, int grid, hipStream_t st) {
    return a.cs_order > 0 ? launch_osd_t<true>(a, W, grid, st) : launch_osd_t<false>(a, W, grid, st);
}

}  // namespace qlsd
