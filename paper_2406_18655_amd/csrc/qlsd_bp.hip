// Min-sum belief propagation, parallel (flooding) schedule, for many shots at once.
//
// Message rules (Hillmann et al., Sec. 4.3: min-sum with scaling alpha, parallel schedule):
//   check -> fault : r_{i->j} = (-1)^{s_i} * alpha * prod_{j' != j} sgn(q_{j'->i}) * min_{j' != j} |q_{j'->i}|
//   fault -> check : q_{j->i} = lambda_j + sum_{i' != i} r_{i'->j},  L_j = lambda_j + sum_i r_{i->j}
//   hard decision  : e_j = [L_j < 0]; a shot has converged once H e = s (tested after every iteration).
// Magnitudes of q and L are clamped to 2^64 so that 100 iterations cannot overflow float32.
//
// Design (MI355X): a workgroup owns S shot "slots" whose messages live entirely in LDS in an
// [edge][slot] layout, so lanes that work on the same check or fault for consecutive slots hit
// consecutive LDS banks.  Each loop iteration runs one check phase and one fault phase over the
// active slots only.  A slot whose shot converged (or ran out of iterations) is retired and
// immediately refilled from a global queue, so early-exiting shots never leave lanes idle; the
// number of work items shrinks only once the queue is empty.  HBM traffic is only the syndrome
// in, the correction out, and the posterior LLRs of shots that go on to LSD.
#include "qlsd_internal.h"

namespace qlsd {

namespace {

constexpr float kClamp = 18446744073709551616.0f;  // 2^64

__device__ __forceinline__ float clampf(float x) { return __builtin_amdgcn_fmed3f(x, -kClamp, kClamp); }

struct BpLds {
    float *msg, *Lv, *lam;
    int *sshot, *siter, *sbad, *act, *ctl, *retk, *newk;
    uint16_t *rp, *ci, *cp, *ce;
    uint8_t *syn;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__device__ inline BpLds carve_bp(unsigned char *base, int m, int n, int E, int S) {
    BpLds L;
    size_t off = 0;
    L.msg = (float *)(base + off); off += sizeof(float) * (size_t)E * S;
    L.Lv = (float *)(base + off); off += sizeof(float) * (size_t)n * S;
    L.lam = (float *)(base + off); off += sizeof(float) * n;
    L.sshot = (int *)(base + off); off += sizeof(int) * S;
    L.siter = (int *)(base + off); off += sizeof(int) * S;
    L.sbad = (int *)(base + off); off += sizeof(int) * S;
    L.act = (int *)(base + off); off += sizeof(int) * S;
    L.retk = (int *)(base + off); off += sizeof(int) * S;
    L.newk = (int *)(base + off); off += sizeof(int) * S;
    L.ctl = (int *)(base + off); off += sizeof(int) * 8;
    L.rp = (uint16_t *)(base + off); off += sizeof(uint16_t) * (m + 1);
    L.ci = (uint16_t *)(base + off); off += sizeof(uint16_t) * E;
    L.cp = (uint16_t *)(base + off); off += sizeof(uint16_t) * (n + 1);
    L.ce = (uint16_t *)(base + off); off += sizeof(uint16_t) * E;
    L.syn = (uint8_t *)(base + off);
    return L;
}

// Walks the flattened (row, active-slot) item space of one phase: item = row * A + a.
struct ItemWalk {
    int row, a, qd, rm, A;
    __device__ ItemWalk(int t, int NT, int A_) : A(A_) {
        row = t / A;
        a = t - row * A;
        qd = NT / A;
        rm = NT - qd * A;
    }
    __device__ __forceinline__ void next() {
        a += rm;
        row += qd;
        if (a >= A) { a -= A; row++; }
    }
};

template <int MAXRW, int MAXCW>
__global__ __launch_bounds__(kBpThreads) void bp_lds_kernel(BpArgs args) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = threadIdx.x, NT = blockDim.x;
    const int m = args.g.m, n = args.g.n, E = args.g.nnz, S = args.S;
    BpLds L = carve_bp(smem, m, n, E, S);

    for (int x = t; x <= m; x += NT) L.rp[x] = (uint16_t)args.g.row_ptr[x];
    for (int x = t; x < E; x += NT) L.ci[x] = (uint16_t)args.g.col_idx[x];
    for (int x = t; x <= n; x += NT) L.cp[x] = (uint16_t)args.g.col_ptr[x];
    for (int x = t; x < E; x += NT) L.ce[x] = (uint16_t)args.g.col_edge[x];
    for (int x = t; x < n; x += NT) L.lam[x] = args.lam[x];
    for (int k = t; k < S; k += NT) { L.sshot[k] = -1; L.siter[k] = 0; L.sbad[k] = 0; }
    __syncthreads();

    const float alpha = args.alpha;
    const int T = args.max_iter;

    for (;;) {
        // ---- slot management: retire converged / exhausted shots, collect slots to refill
        if (t == 0) { L.ctl[0] = 0; L.ctl[1] = 0; }
        __syncthreads();
        if (t < S) {
            const int k = t;
            bool need = L.sshot[k] < 0;
            if (!need) {
                const int it = L.siter[k];
                const bool conv = it >= 1 && !L.sbad[k];
                if ((args.early_exit && conv) || it >= T) {
                    L.retk[atomicAdd(&L.ctl[0], 1)] = k;
                    need = true;
                } else {
                    L.sbad[k] = 0;
                }
            }
            if (need) L.newk[atomicAdd(&L.ctl[1], 1)] = k;
        }
        __syncthreads();
        if (t == 0) {
            const int want = L.ctl[1];
            L.ctl[2] = want ? atomicAdd(args.next_shot, want) : 0;
        }
        __syncthreads();
        const int nret = L.ctl[0], nnew = L.ctl[1], base = L.ctl[2];

        // ---- outputs of retired shots (coalesced rows)
        for (int r = 0; r < nret; r++) {
            const int k = L.retk[r];
            const int shot = L.sshot[k];
            const int it = L.siter[k];
            const bool conv = it >= 1 && !L.sbad[k];
            const size_t row = (size_t)shot * n;
            for (int j = t; j < n; j += NT) {
                const float Lj = L.Lv[j * S + k];
                if (args.corr) args.corr[row + j] = Lj < 0.f ? 1 : 0;
                if (args.llr_out) args.llr_out[row + j] = Lj;
                if (!conv && args.llr_lsd) args.llr_lsd[row + j] = Lj;
            }
            if (t == 0) {
                if (args.info) {
                    qlsd_shot_info inf;
                    inf.status = conv ? QLSD_ST_BP_CONVERGED : 0;
                    inf.reserved = 0;
                    inf.bp_iters = (int16_t)it;
                    inf.n_clusters = 0;
                    inf.rounds = 0;
                    inf.max_cluster_cols = 0;
                    args.info[shot] = inf;
                }
                if (!conv && args.lsd_list) args.lsd_list[atomicAdd(args.lsd_count, 1)] = shot;
            }
        }
        __syncthreads();

        // ---- refill: syndrome in, c->v messages zero (the next fault phase then sets q = lambda)
        for (int r = 0; r < nnew; r++) {
            const int k = L.newk[r];
            const int shot = base + r;
            const bool valid = shot < args.B;
            if (t == 0) { L.sshot[k] = valid ? shot : -1; L.siter[k] = -1; L.sbad[k] = 0; }
            if (valid) {
                const uint8_t *s = args.syn + (size_t)shot * m;
                for (int i = t; i < m; i += NT) L.syn[i * S + k] = s[i] & 1;
                for (int e = t; e < E; e += NT) L.msg[e * S + k] = 0.f;
            }
        }
        __syncthreads();
        if (t == 0) {
            int na = 0;
            for (int k = 0; k < S; k++)
                if (L.sshot[k] >= 0) L.act[na++] = k;
            L.ctl[3] = na;
        }
        __syncthreads();
        const int A = L.ctl[3];
        if (A == 0) break;

        // ---- fault (variable-node) phase: L = lambda + sum r, q = exclusive sums
        {
            ItemWalk w(t, NT, A);
            for (int idx = t; idx < n * A; idx += NT, w.next()) {
                const int j = w.row, k = L.act[w.a];
                const int c0 = L.cp[j], cw = L.cp[j + 1] - c0;
                float r[MAXCW];
                int eid[MAXCW];
#pragma unroll
                for (int u = 0; u < MAXCW; u++) {
                    if (u < cw) {
                        eid[u] = L.ce[c0 + u];
                        r[u] = L.msg[eid[u] * S + k];
                    }
                }
                const float lam = L.lam[j];
                float pre[MAXCW + 1];
                pre[0] = lam;
#pragma unroll
                for (int u = 0; u < MAXCW; u++) pre[u + 1] = (u < cw) ? pre[u] + r[u] : pre[u];
                float suf = 0.f;
#pragma unroll
                for (int u = MAXCW - 1; u >= 0; u--) {
                    if (u < cw) {
                        const float q = (u + 1 < cw) ? pre[u] + suf : pre[u];
                        L.msg[eid[u] * S + k] = clampf(q);
                        suf = (u + 1 < cw) ? r[u] + suf : r[u];
                    }
                }
                float Lt = lam;
#pragma unroll
                for (int u = 0; u < MAXCW; u++)
                    if (u < cw) Lt = pre[u + 1];
                L.Lv[j * S + k] = clampf(Lt);
            }
        }
        __syncthreads();
        if (t < A) L.siter[L.act[t]] += 1;
        __syncthreads();

        // ---- check phase: min-sum messages; syndrome test of the current hard decision
        {
            ItemWalk w(t, NT, A);
            for (int idx = t; idx < m * A; idx += NT, w.next()) {
                const int i = w.row, k = L.act[w.a];
                const int e0 = L.rp[i], rw = L.rp[i + 1] - e0;
                const bool test = L.siter[k] >= 1;
                const uint32_t sb = L.syn[i * S + k];
                uint32_t sg = sb << 31;
                uint32_t hp = 0;
                float mn1 = INFINITY, mn2 = INFINITY;
                float q[MAXRW];
#pragma unroll
                for (int u = 0; u < MAXRW; u++) {
                    if (u < rw) {
                        const int e = e0 + u;
                        q[u] = L.msg[e * S + k];
                        sg ^= __float_as_uint(q[u]);
                        const float a = fabsf(q[u]);
                        mn2 = __builtin_amdgcn_fmed3f(mn1, mn2, a);
                        mn1 = fminf(mn1, a);
                        if (test) hp ^= L.Lv[L.ci[e] * S + k] < 0.f ? 1u : 0u;
                    }
                }
                if (test && hp != sb) L.sbad[k] = 1;
                const float m1 = alpha * mn1, m2 = alpha * mn2;
#pragma unroll
                for (int u = 0; u < MAXRW; u++) {
                    if (u < rw) {
                        const float mag = (fabsf(q[u]) == mn1) ? m2 : m1;
                        const uint32_t sgn = (sg ^ __float_as_uint(q[u])) & 0x80000000u;
                        L.msg[(e0 + u) * S + k] = __uint_as_float(__float_as_uint(mag) | sgn);
                    }
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace

size_t bp_lds_bytes(const DevGraph &g, int S) {
    size_t b = 0;
    b += sizeof(float) * ((size_t)g.nnz * S + (size_t)g.n * S + g.n);
    b += sizeof(int) * (6 * (size_t)S + 8);
    b += sizeof(uint16_t) * ((size_t)g.m + 1 + g.nnz + g.n + 1 + g.nnz);
    b += (size_t)g.m * S;
    return align16(b);
}

template <int RW, int CW>
static hipError_t launch_bp_t(const BpArgs &a, int grid, size_t lds, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)bp_lds_kernel<RW, CW>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((bp_lds_kernel<RW, CW>), dim3(grid), dim3(kBpThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_bp(const BpArgs &a, int grid, hipStream_t st) {
    const size_t lds = bp_lds_bytes(a.g, a.S);
    if (a.g.max_rw <= 8 && a.g.max_cw <= 4) return launch_bp_t<8, 4>(a, grid, lds, st);
    if (a.g.max_rw <= 16 && a.g.max_cw <= 8) return launch_bp_t<16, 8>(a, grid, lds, st);
    return launch_bp_t<kMaxRowWeight, kMaxColWeight>(a, grid, lds, st);
}

namespace {
__global__ void zero_kernel(int *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}
}  // namespace

hipError_t launch_zero(int *p, int count, hipStream_t st) {
    hipLaunchKernelGGL(zero_kernel, dim3((count + 255) / 256), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

}  // namespace qlsd
