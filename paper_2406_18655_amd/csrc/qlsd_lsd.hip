// Localized statistics decoding (LSD-0) on the GPU: one wavefront per shot.
//
// What is computed (Hillmann et al., Sec. 4.1 / Alg. 1, Defs. 4.1-4.4, with the synchronous
// rounds of Appendix B / Alg. 2):
//   * one cluster per flipped detector;
//   * per round, every invalid cluster C picks its candidate fault of lowest key (llr_j, j)
//     among Lambda(C) = N(checks(C)) \ faults(C), all picks made on the round-start state;
//   * the picked faults join their clusters; clusters that own, or in this round claim, a
//     common detector of a picked fault merge (Def. 4.4);
//   * the new columns are reduced on the fly (Sec. 4.2), in ascending key order, and a cluster
//     is valid once its local syndrome lies in the image of its columns;
//   * once every cluster is valid, each is solved on its pivot columns and the union is e_hat.
//
// MI355X mapping.  A shot's clusters own disjoint detector sets, so the elimination of all its
// clusters can share one row space: detectors get compact "local rows" in the order they join a
// cluster, and all reductions happen in a single Gauss-Jordan basis over those rows.  Columns of
// different clusters never share a row, so this is exactly the block-diagonal form that the
// paper's merge step (Sec. 4.2, block swap of zero rows) produces -- a merge costs nothing.
// The basis is bit-sliced across the wavefront: lane l holds local rows l, l+64, ... and, for
// each, the row's bits over the pivot rows (Mrow) and, for the column that created each pivot,
// the pivots whose combination contains it (CT).  Reducing a new column, adding a pivot and
// solving are then per-lane AND/XOR/popcount plus a few ballots -- no cross-lane reductions.
// Union-find over local rows lives in LDS (lock-free CAS hooking of the larger root under the
// smaller one); candidate selection is a per-row scan plus an LDS 64-bit atomic min per root.
#include "qlsd_lsd_dev.h"

namespace qlsd {

namespace {

// At most 128 VGPRs (4 wavefronts per SIMD) for W <= 2, 256 (2 per SIMD) for W = 4.  CB: the
// cluster-batched schedule of the column insertion (W = 4 only; chosen by the autotuner).
template <int W, bool GL, bool MU, bool CB = false>
__global__ __launch_bounds__(kLsdThreads) __attribute__((amdgpu_waves_per_eu(W <= 2 ? 4 : 2)))
void lsd_kernel(LsdArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    constexpr int K = 64 * W;
    // after the fused kernel: nothing to do when every published shot was decoded there
    if (A.skip_done && A.done_count && *A.done_count >= *A.list_count) return;
    const int m = A.g.m, n = A.g.n, E = A.g.nnz;
    GView<GL> g;
    g.max_cw = A.g.max_cw;
    size_t gbytes = 0;
    if constexpr (GL) {
        uint16_t *t16 = (uint16_t *)smem;
        uint16_t *rp = t16, *ci = rp + (m + 1), *cp = ci + E, *ri = cp + (n + 1);
        for (int x = threadIdx.x; x <= m; x += blockDim.x) rp[x] = (uint16_t)A.g.row_ptr[x];
        for (int x = threadIdx.x; x < E; x += blockDim.x) ci[x] = (uint16_t)A.g.col_idx[x];
        for (int x = threadIdx.x; x <= n; x += blockDim.x) cp[x] = (uint16_t)A.g.col_ptr[x];
        for (int x = threadIdx.x; x < E; x += blockDim.x) ri[x] = (uint16_t)A.g.row_idx[x];
        g.rp = rp; g.ci = ci; g.cp = cp; g.ri = ri;
        gbytes = lsd_graph_bytes(m, n, E);
        __syncthreads();
    } else {
        g.rp = A.g.row_ptr; g.ci = A.g.col_idx; g.cp = A.g.col_ptr; g.ri = A.g.row_idx;
    }
    unsigned char *base = smem + gbytes + (size_t)wid * A.wave_bytes;
    const LsdLds S = carve_lsd(base, m, n, K, A.keys_in_lds != 0, A.mu > 0);

    const int total = A.list ? *A.list_count : A.count;
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(A.next_item, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= total) break;
        const int shot = A.list ? A.list[item] : item;
        if (A.skip_done && shot < 0) continue;
        decode_shot<W, MU, GView<GL>, false, true, false, CB>(A, S, g, shot, lane);
        wave_sync();
    }
}

template <int W, bool GL, bool MU, bool CB>
hipError_t launch_lsd_k(const LsdArgs &a, int grid, size_t lds, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)lsd_kernel<W, GL, MU, CB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((lsd_kernel<W, GL, MU, CB>), dim3(grid), dim3(kLsdThreads), lds, st, a);
    return hipGetLastError();
}

template <int W, bool MU>
hipError_t launch_lsd_w(const LsdArgs &a, int grid, hipStream_t st) {
    const size_t lds = (a.graph_in_lds ? lsd_graph_bytes(a.g.m, a.g.n, a.g.nnz) : 0) +
                       (size_t)a.wave_bytes * (kLsdThreads / 64);
    if constexpr (W == 4) {
        if (a.cluster_batched)
            return a.graph_in_lds ? launch_lsd_k<W, true, MU, true>(a, grid, lds, st)
                                  : launch_lsd_k<W, false, MU, true>(a, grid, lds, st);
    }
    return a.graph_in_lds ? launch_lsd_k<W, true, MU, false>(a, grid, lds, st)
                          : launch_lsd_k<W, false, MU, false>(a, grid, lds, st);
}

// Overflow LSD for the shots whose clusters outgrew the register basis of lsd_kernel (listed by
// it): one wavefront per workgroup runs the same per-shot code with 64 WW local rows, visiting
// only the slices of local rows in use.  Shots beyond the last tier keep the OVERFLOW status.
// BLDS (WW = kMidW): the basis sits in LDS after the wavefront's arrays, and a shot that outgrows
// it is listed for the device-memory kernel (A.ovf_list); otherwise (WW = kWideW) the basis is the
// workgroup's block of ws.
template <bool MU, int WW, bool BLDS>
__global__ __launch_bounds__(64) void lsd_wide_kernel(LsdArgs A, uint64_t *ws) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int total = *A.list_count;
    if (total == 0) return;
    GView<false> g;
    g.max_cw = A.g.max_cw;
    g.rp = A.g.row_ptr; g.ci = A.g.col_idx; g.cp = A.g.col_ptr; g.ri = A.g.row_idx;
    size_t offs[kLsdLayoutEntries];
    const size_t arrays = lsd_layout(A.g.m, A.g.n, 64 * WW, A.keys_in_lds != 0, A.mu > 0, offs, kWideDependent);
    const LsdLds S = carve_lsd(smem, A.g.m, A.g.n, 64 * WW, A.keys_in_lds != 0, A.mu > 0, kWideDependent);
    uint64_t *mem = BLDS ? (uint64_t *)(smem + ((arrays + 15) & ~(size_t)15))
                         : ws + (size_t)blockIdx.x * (2 * WW * WW * 64);
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(A.next_item, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= total) break;
        decode_shot<WW, MU, GView<false>, true, BLDS, BLDS>(A, S, g, A.list[item], lane, mem);
        wave_sync();
    }
}

// Optimal factorization (Appendix A) of each error: connected components of its faults in the
// fault graph.  One wavefront per shot (grid-stride): every detector of a faulty column remembers
// the first faulty column that reached it and unites later ones with it (lock-free hooking of
// the larger root under the smaller, as in LSD); then each component's size is counted at its root.
__global__ __launch_bounds__(64) void error_cluster_kernel(DevGraph g, const uint8_t *e, int B,
                                                           qlsd_cluster_stats *out) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x;
    const int m = g.m, n = g.n;
    int32_t *par = (int32_t *)smem;   // n
    int32_t *cnt = par + n;           // n
    int32_t *owner = cnt + n;         // m
    for (int b = blockIdx.x; b < B; b += gridDim.x) {
        const uint8_t *er = e + (size_t)b * n;
        for (int j = lane; j < n; j += 64) { par[j] = j; cnt[j] = 0; }
        for (int i = lane; i < m; i += 64) owner[i] = -1;
        wave_sync();
        for (int j = lane; j < n; j += 64) {
            if (!(er[j] & 1)) continue;
            for (int k = g.col_ptr[j]; k < g.col_ptr[j + 1]; k++) {
                const int prev = atomicCAS(&owner[g.row_idx[k]], -1, j);
                if (prev >= 0) unite(par, prev, j);
            }
        }
        wave_sync();
        for (int j = lane; j < n; j += 64)
            if (er[j] & 1) atomicAdd(&cnt[find_root(par, j)], 1);
        wave_sync();
        uint32_t nu = 0u, mx = 0u, tot = 0u, sq = 0u;
        for (int j = lane; j < n; j += 64) {
            const uint32_t v = (uint32_t)cnt[j];
            nu += v ? 1u : 0u;
            mx = v > mx ? v : mx;
            tot += v;
            sq += v * v;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            nu += (uint32_t)__shfl_xor((int)nu, off, 64);
            const uint32_t o = (uint32_t)__shfl_xor((int)mx, off, 64);
            mx = o > mx ? o : mx;
            tot += (uint32_t)__shfl_xor((int)tot, off, 64);
            sq += (uint32_t)__shfl_xor((int)sq, off, 64);
        }
        if (lane == 0) out[b] = qlsd_cluster_stats{(int)nu, (int)mx, (int)tot, (int)sq};
        wave_sync();
    }
}

// Shots flagged by BP -> a dense list (one 64-shot ballot and one atomic per wavefront).
// Lists the flagged shots.  A 256-thread workgroup takes 1024 consecutive flags, four per thread
// (one 32-bit read when the flags are 4-byte aligned), counts them with a wavefront scan, reserves
// its whole share of the list with a single atomic and writes its entries in shot order: one
// atomic per 1024 shots instead of one per 64 (the per-wavefront form spent most of its 13 us per
// 65,536-shot batch queued on that counter).  The order of entries across workgroups is the order
// of their atomics; every consumer decodes the listed shots independently.
constexpr int kCompactPerThread = 4;
constexpr int kCompactPerBlock = 256 * kCompactPerThread;
__global__ __launch_bounds__(256) void compact_kernel(const uint8_t *flag, int B, int *list, int *count) {
    __shared__ int wsum[4];
    __shared__ int wgbase;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int b0 = blockIdx.x * kCompactPerBlock + t * kCompactPerThread;
    uint32_t bits = 0;  // bit k: shot b0 + k is flagged
    if (b0 + kCompactPerThread <= B && (((uintptr_t)flag) & 3) == 0) {
        const uint32_t w = *(const uint32_t *)(flag + b0);
#pragma unroll
        for (int k = 0; k < kCompactPerThread; k++) bits |= (((w >> (8 * k)) & 0xffu) != 0u ? 1u : 0u) << k;
    } else {
#pragma unroll
        for (int k = 0; k < kCompactPerThread; k++) bits |= (b0 + k < B && flag[b0 + k] ? 1u : 0u) << k;
    }
    const int c = __popc(bits);
    int incl = c;  // inclusive scan over the wavefront
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    if (t == 0) {
        const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        wgbase = total > 0 ? atomicAdd(count, total) : 0;
    }
    __syncthreads();
    int pos = wgbase + incl - c;
    for (int w = 0; w < wave; w++) pos += wsum[w];
#pragma unroll
    for (int k = 0; k < kCompactPerThread; k++)
        if ((bits >> k) & 1u) list[pos++] = b0 + k;
}

}  // namespace

hipError_t launch_compact(const uint8_t *flag, int B, int *list, int *count, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(compact_kernel, dim3((B + kCompactPerBlock - 1) / kCompactPerBlock), dim3(256), 0, st, flag, B,
                       list, count);
    return hipGetLastError();
}

size_t lsd_wave_bytes(const DevGraph &g, int W, bool keys_in_lds, bool with_mu) {
    size_t offs[kLsdLayoutEntries];
    return lsd_layout(g.m, g.n, 64 * W, keys_in_lds, with_mu, offs);
}

size_t lsd_total_lds(const DevGraph &g, int W, bool keys_in_lds, bool graph_in_lds, bool with_mu) {
    return (graph_in_lds ? lsd_graph_bytes(g.m, g.n, g.nnz) : 0) +
           lsd_wave_bytes(g, W, keys_in_lds, with_mu) * (kLsdThreads / 64);
}

hipError_t launch_error_clusters(const DevGraph &g, const uint8_t *e, int B, qlsd_cluster_stats *out, hipStream_t st) {
    const size_t lds = sizeof(int32_t) * (2 * (size_t)g.n + g.m);
    hipError_t err = hipFuncSetAttribute((const void *)error_cluster_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    const int grid = B < 4096 ? B : 4096;
    hipLaunchKernelGGL(error_cluster_kernel, dim3(grid), dim3(64), lds, st, g, e, B, out);
    return hipGetLastError();
}

size_t lsd_wide_ws_words() { return (size_t)2 * kWideW * kWideW * 64; }

size_t lsd_wide_lds(const DevGraph &g, bool keys_in_lds, bool with_mu) {
    size_t offs[kLsdLayoutEntries];
    return lsd_layout(g.m, g.n, kWideRows, keys_in_lds, with_mu, offs, kWideDependent);
}

size_t lsd_mid_lds(const DevGraph &g, bool keys_in_lds, bool with_mu) {
    size_t offs[kLsdLayoutEntries];
    const size_t arrays = lsd_layout(g.m, g.n, kMidRows, keys_in_lds, with_mu, offs, kWideDependent);
    return ((arrays + 15) & ~(size_t)15) + sizeof(uint64_t) * 2 * kMidW * kMidW * 64;
}

template <bool MU, int WW, bool BLDS>
static hipError_t launch_wide_t(const LsdArgs &a, uint64_t *ws, int grid, size_t lds, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)lsd_wide_kernel<MU, WW, BLDS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((lsd_wide_kernel<MU, WW, BLDS>), dim3(grid), dim3(64), lds, st, a, ws);
    return hipGetLastError();
}

hipError_t launch_lsd_wide(const LsdArgs &a, uint64_t *ws, int grid, hipStream_t st) {
    const size_t lds = lsd_wide_lds(a.g, a.keys_in_lds != 0, a.mu > 0);
    return a.mu > 0 ? launch_wide_t<true, kWideW, false>(a, ws, grid, lds, st)
                    : launch_wide_t<false, kWideW, false>(a, ws, grid, lds, st);
}

hipError_t launch_lsd_mid(const LsdArgs &a, int grid, hipStream_t st) {
    const size_t lds = lsd_mid_lds(a.g, a.keys_in_lds != 0, a.mu > 0);
    return a.mu > 0 ? launch_wide_t<true, kMidW, true>(a, nullptr, grid, lds, st)
                    : launch_wide_t<false, kMidW, true>(a, nullptr, grid, lds, st);
}

// LSD-mu decoders always use W = 4 (their extra growth rounds need the room), so LSD-mu code is
// instantiated for W = 4 only.
hipError_t launch_lsd(const LsdArgs &a, int W, int grid, hipStream_t st) {
    if (a.mu > 0) return W == 4 ? launch_lsd_w<4, true>(a, grid, st) : hipErrorInvalidValue;
    switch (W) {
        case 1: return launch_lsd_w<1, false>(a, grid, st);
        case 2: return launch_lsd_w<2, false>(a, grid, st);
        case 4: return launch_lsd_w<4, false>(a, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace qlsd
