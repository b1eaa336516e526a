// Per-shot LSD device code (one wavefront per shot), shared by the stand-alone LSD kernel and the
// fused BP + LSD kernel.  What it computes and how it maps onto the wavefront is described at
// the top of qlsd_lsd.hip.
#pragma once
#include <type_traits>

#include "qlsd_internal.h"

namespace qlsd {

namespace {


__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// A wave-uniform 64-bit value, kept in scalar registers.  The compiler cannot always prove that
// values updated across the LSD round loop stay uniform and then keeps them in vector registers,
// where every test on them costs vector instructions.
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint32_t lo = __shfl_xor((int)(uint32_t)v, off, 64);
        const uint32_t hi = __shfl_xor((int)(uint32_t)(v >> 32), off, 64);
        const uint64_t o = ((uint64_t)hi << 32) | lo;
        v = o < v ? o : v;
    }
    return v;
}

// Order-preserving map of a float32 LLR to uint32 (-0 treated as +0).
__device__ __forceinline__ uint32_t ordered_key(float x) {
    uint32_t u = __float_as_uint(x);
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Read-only view of H used by the LSD kernel: u16 copies in LDS (small codes) or the int32
// arrays in global memory.
template <bool InLds>
struct GView {
    static constexpr bool kInLds = InLds;  // graph in LDS implies keys in LDS (the host's placement rule)
    using T = typename std::conditional<InLds, uint16_t, int32_t>::type;
    const T *rp, *ci, *cp, *ri;
    int max_cw;
    __device__ __forceinline__ int row_ptr(int i) const { return rp[i]; }
    __device__ __forceinline__ int col_idx(int e) const { return ci[e]; }
    __device__ __forceinline__ int col_ptr(int j) const { return cp[j]; }
    __device__ __forceinline__ int row_idx(int e) const { return ri[e]; }
};

constexpr int kFree = 0x7fffffff;
constexpr int kMaxMu = 12;  // largest supported order mu (2^mu patterns per cluster)
constexpr uint8_t kValid = 0, kInvalid = 1, kFrozen = 2;
constexpr int kBatchMin = 4;  // cluster-batched schedule: selections in a round from which it batches

struct LsdLds {
    uint32_t *keys;    // n (when keys_in_lds)
    uint64_t *sel;     // K: per-root best candidate key
    uint64_t *lkey;    // K: selection list keys
    int32_t *lroot;    // K: selection list roots
    int32_t *colAt;    // K: column that created the pivot at this local row
    int32_t *croot;    // K: union-find parent over local rows
    int32_t *rowOf;    // K: detector of each local row
    int32_t *loc;      // m: local row of each detector, -1 if unclustered
    int32_t *claimer;  // m: smallest root claiming an unclustered detector this round
    uint32_t *incol;   // ceil(n/32): fault already in a cluster
    uint8_t *state;    // K: kValid / kInvalid / kFrozen (meaningful at roots)
    int32_t *ctl;      // 4: [0] local row count
    int32_t *colNP;    // KNP: clustered columns that were dependent when added (LSD-mu)
    int64_t *wq;       // K: integer weight of the column that created each pivot (LSD-mu)
    uint64_t *zk;      // kMaxMu * W: solution change of each reprocessed column (LSD-mu)
    int32_t *tsel;     // kMaxMu: reprocessed columns of the current cluster (LSD-mu)
    int64_t *tw;       // kMaxMu: their weights
    uint64_t *cand;    // K: cached smallest candidate key of each local row (kStale: recompute)
    uint32_t *cbit;    // ceil(n/32): the correction, one bit per fault (the row is written once)
};

// A row's cached candidate stays exact while its column is not taken: the taken set only grows,
// so the minimum over the row's remaining faults can change only when that column is taken.  The
// rows that may cache a column are its own detectors, all local rows by the time it is taken, so
// taking a column marks exactly those rows kStale and the selection never tests the cached column.
constexpr uint64_t kStale = ~0ull - 1ull;

__host__ __device__ inline size_t align8(size_t x) { return (x + 7) & ~size_t(7); }

constexpr int kLsdLayoutEntries = 19;

// Arrays sized by K (a compile-time constant in the kernels) and by fixed constants come first, so
// their offsets from the wavefront's block are constants the compiler folds into the LDS
// instructions (no register per array); 8-byte arrays before 4-byte ones before bytes keeps every
// array aligned.  The arrays sized by m and n follow.  offs[] keeps the field order of LsdLds.
// with_mu: room for the LSD-mu arrays (wq, zk, tw, colNP, tsel); LSD-0 never touches them.
// knp: entries of colNP (0: K).
__host__ __device__ inline size_t lsd_layout(int m, int n, int K, bool keys_in_lds, bool with_mu, size_t *offs,
                                             int knp = 0) {
    if (knp <= 0) knp = K;
    const size_t mu = with_mu ? 1 : 0;
    size_t off = 0;
    offs[1] = off; off += sizeof(uint64_t) * K;                      // sel
    offs[2] = off; off += sizeof(uint64_t) * K;                      // lkey
    offs[17] = off; off += sizeof(uint64_t) * K;                     // cand
    offs[13] = off; off += mu * sizeof(int64_t) * K;                 // wq
    offs[14] = off; off += mu * sizeof(uint64_t) * kMaxMu * (K / 64);// zk
    offs[16] = off; off += mu * sizeof(int64_t) * kMaxMu;            // tw
    offs[3] = off; off += sizeof(int32_t) * K;                       // lroot
    offs[4] = off; off += sizeof(int32_t) * K;                       // colAt
    offs[5] = off; off += sizeof(int32_t) * K;                       // croot
    offs[6] = off; off += sizeof(int32_t) * K;                       // rowOf
    offs[12] = off; off += mu * sizeof(int32_t) * knp;               // colNP
    offs[15] = off; off += mu * sizeof(int32_t) * kMaxMu;            // tsel
    offs[11] = off; off += sizeof(int32_t) * 4;                      // ctl
    offs[10] = off; off += align8(K);                                // state
    offs[0] = off; off += keys_in_lds ? sizeof(uint32_t) * n : 0;    // keys
    offs[7] = off; off += sizeof(int32_t) * m;                       // loc
    offs[8] = off; off += sizeof(int32_t) * m;                       // claimer
    offs[9] = off; off += sizeof(uint32_t) * ((n + 31) / 32);        // incol
    offs[18] = off; off += sizeof(uint32_t) * ((n + 31) / 32);       // cbit
    return align8(off);
}

__host__ __device__ inline size_t lsd_graph_bytes(int m, int n, int nnz) {
    return align8(sizeof(uint16_t) * ((size_t)m + 1 + nnz + n + 1 + nnz));
}

// Union-find parents live in LDS and other lanes hook roots concurrently, so every read goes to
// LDS (volatile); the LDS-qualified pointer keeps those reads ds_read instructions (a generic
// volatile pointer compiles to flat loads, which also wait on the vector-memory counter).
typedef __attribute__((address_space(3))) int32_t lds_int32;
__device__ __forceinline__ int parent_of(const int32_t *par, int x) {
    return ((const volatile lds_int32 *)par)[x];
}
__device__ __forceinline__ int find_root(const int32_t *par, int x) {
    int p = parent_of(par, x);
    while (p != x) { x = p; p = parent_of(par, x); }
    return x;
}

// Returns true iff it hooked one root under another (false: already in one set).
__device__ bool unite(int32_t *par, int x, int y) {
    for (;;) {
        x = find_root(par, x);
        y = find_root(par, y);
        if (x == y) return false;
        if (x < y) { const int tmp = x; x = y; y = tmp; }
        // hook the larger root under the smaller one
        if (atomicCAS(&par[x], x, y) == x) return true;
    }
}

// The shot's Gauss-Jordan basis.  Mrow(s, w): lane row s's bits over pivot local rows 64w..64w+63
// (rows of the reduced pivot vectors); CT(s, w): for a pivot row, the pivots whose combination uses
// the column that created it.  InMem = false keeps both in registers (the LSD kernels, W <= 4);
// InMem = true keeps them in a per-wavefront block of memory ([2][W][W][64] words, lane fastest)
// for the kernels that take the shots whose clusters outgrow the register basis: in LDS (InLds,
// the 512-row kernel) or in device memory (the 1024-row kernel).
typedef __attribute__((address_space(3))) uint64_t lds_u64;

template <int W, bool InMem, bool InLds = false>
struct Basis;

template <int W>
struct Basis<W, false, false> {
    uint64_t Mrow[W][W];
    uint64_t CT[W][W];
    uint64_t piv[W];  // uniform: pivot local rows
    uint64_t sp[W];   // uniform: reduced syndrome over local rows
    int ns;           // uniform: slices 0..ns-1 of local rows are in use (the rest stays zero)
    static constexpr bool kInMem = false;
    __device__ __forceinline__ uint64_t &M(int s, int w) { return Mrow[s][w]; }
    __device__ __forceinline__ uint64_t &C(int s, int w) { return CT[s][w]; }
    __device__ __forceinline__ uint64_t M(int s, int w) const { return Mrow[s][w]; }
    __device__ __forceinline__ uint64_t C(int s, int w) const { return CT[s][w]; }
    // slice s of local rows (or of pivot rows) may be non-zero; the register code bounds its
    // loops at compile time instead (insert_column picks a tier from ns)
    __device__ __forceinline__ bool active(int) const { return true; }
    // word w of Mrow at lane row (64 rs + rl), rs < NS; rs is wave-uniform but not a compile-time
    // index, so it is selected by unrolled compares (a runtime array index would put the basis in
    // scratch memory)
    template <int NS = W>
    __device__ __forceinline__ uint64_t row_word(int rs, int w, int rl) const {
        uint64_t v = 0;
#pragma unroll
        for (int s = 0; s < NS; s++)
            if (s == rs) v = readlane64(Mrow[s][w], rl);
        return v;
    }
};

template <int W, bool InLds>
struct Basis<W, true, InLds> {
    // an LDS-qualified pointer keeps the accesses ds_ instructions
    using Ptr = typename std::conditional<InLds, lds_u64 *, uint64_t *>::type;
    Ptr mem;        // this wavefront's block, offset by its lane
    int ns;         // uniform: slices 0..ns-1 of local rows are in use
    uint64_t piv[W];
    uint64_t sp[W];
    static constexpr bool kInMem = true;
    __device__ __forceinline__ auto &M(int s, int w) { return mem[(s * W + w) * 64]; }
    __device__ __forceinline__ auto &C(int s, int w) { return mem[((W + s) * W + w) * 64]; }
    __device__ __forceinline__ uint64_t M(int s, int w) const { return mem[(s * W + w) * 64]; }
    __device__ __forceinline__ uint64_t C(int s, int w) const { return mem[((W + s) * W + w) * 64]; }
    __device__ __forceinline__ bool active(int s) const { return s < ns; }
    template <int NS = W>
    __device__ __forceinline__ uint64_t row_word(int rs, int w, int rl) const {
        return readlane64(mem[(rs * W + w) * 64], rl);
    }
};

template <int W>
__device__ __forceinline__ int parity_and(const uint64_t (&a)[W], const uint64_t (&b)[W]) {
    int c = 0;
#pragma unroll
    for (int w = 0; w < W; w++) c += __popcll(a[w] & b[w]);
    return c & 1;
}

// parity of (row s of Mrow, or of CT) AND b over the slices in use (the first NS)
template <int W, class BB, int NS = W>
__device__ __forceinline__ int parity_M(const BB &B, int s, const uint64_t (&b)[W]) {
    int c = 0;
#pragma unroll
    for (int w = 0; w < NS; w++)
        if (B.active(w)) c += __popcll(B.M(s, w) & b[w]);
    return c & 1;
}
template <int W, class BB, int NS = W>
__device__ __forceinline__ int parity_C(const BB &B, int s, const uint64_t (&b)[W]) {
    int c = 0;
#pragma unroll
    for (int w = 0; w < NS; w++)
        if (B.active(w)) c += __popcll(B.C(s, w) & b[w]);
    return c & 1;
}

// Adds column col (its detectors are all clustered) to the Gauss-Jordan basis.  Returns true iff
// it became a pivot.  On-the-fly elimination (Sec. 4.2): only the new column is reduced.
// The column's local rows are held by lanes base .. base + cw - 1 of lr_src (-1: no entry).
// Two steps: the reduction of the column against the basis (insert_plan, which only reads the
// basis) and the update of the basis with the new pivot (insert_apply).
template <int W>
struct InsertPlan {
    uint32_t bpf;    // this lane: bit s = local row 64 s + lane lies in the reduced column
    uint32_t cflag;  // this lane: bit s = pivot row 64 s + lane's combination uses the column
    uint64_t bp[W];  // uniform: the reduced column over local rows
    uint64_t R[W];   // uniform: the new pivot row's Mrow words
    int rs, rl;      // uniform: the new pivot's local row, 64 rs + rl
};

// NS: only local-row slices 0..NS-1 can be non-zero (the shot's rows all lie below 64 NS), so
// the column, the reduced rows and the new pivot lie there too and the loops stop at NS; the
// entries of P for slices NS..W-1 are zero.  Returns false iff the column is dependent.
template <int W, int NS, class BB>
__device__ __forceinline__ bool insert_plan(const BB &B, int lane, int lr_src, int base, int cw, InsertPlan<W> &P) {
    // the column's support over local rows, as NS wave-uniform masks
    uint64_t cm[W];
#pragma unroll
    for (int s = 0; s < W; s++) cm[s] = 0;
    for (int u = 0; u < cw; u++) {
        const int lr = __builtin_amdgcn_readlane(lr_src, base + u);
        if (lr >= 0 && lr < 64 * NS) {
#pragma unroll
            for (int s = 0; s < NS; s++)
                if ((lr >> 6) == s) cm[s] |= 1ull << (lr & 63);
        }
    }
    uint32_t bf = 0;  // bit s: this lane's local row s*64+lane is in the column's support
#pragma unroll
    for (int s = 0; s < NS; s++) bf |= (uint32_t)((cm[s] >> lane) & 1ull) << s;
    uint64_t a[W];    // the column's support on pivot rows
#pragma unroll
    for (int s = 0; s < W; s++) a[s] = s < NS ? cm[s] & B.piv[s] : 0ull;
    P.bpf = 0;
#pragma unroll
    for (int s = 0; s < NS; s++)
        if (B.active(s)) P.bpf |= (uint32_t)(((bf >> s) & 1u) ^ parity_M<W, BB, NS>(B, s, a)) << s;
    P.rs = -1;
#pragma unroll
    for (int s = 0; s < W; s++) {
        P.bp[s] = s < NS ? ballot((P.bpf >> s) & 1u) : 0ull;
        if (P.rs < 0 && P.bp[s]) P.rs = s;
    }
    if (P.rs < 0) return false;
    uint64_t bprs = 0;
#pragma unroll
    for (int s = 0; s < NS; s++)
        if (s == P.rs) bprs = P.bp[s];
    P.rl = __builtin_ctzll(bprs);
#pragma unroll
    for (int w = 0; w < W; w++) P.R[w] = (w < NS && B.active(w)) ? B.template row_word<NS>(P.rs, w, P.rl) : 0ull;
    P.cflag = 0;
#pragma unroll
    for (int s = 0; s < NS; s++) {
        if (!B.active(s)) continue;
        const bool is_piv = (B.piv[s] >> lane) & 1ull;
        if (is_piv && parity_C<W, BB, NS>(B, s, a)) P.cflag |= 1u << s;
    }
    return true;
}

template <int W, class BB>
__device__ __forceinline__ void insert_apply(BB &B, const LsdLds &S, int col, int lane, const InsertPlan<W> &P) {
    const int rs = P.rs, rl = P.rl;
    // rows in the reduced column's support: eliminate the new pivot row from the old pivots
#pragma unroll
    for (int s = 0; s < W; s++) {
        if ((P.bpf >> s) & 1u) {
#pragma unroll
            for (int w = 0; w < W; w++)
                if (B.active(w)) B.M(s, w) ^= P.R[w] ^ ((w == rs) ? (1ull << rl) : 0ull);
        }
    }
    // combination tracking
#pragma unroll
    for (int s = 0; s < W; s++) {
        if ((P.cflag >> s) & 1u) {
#pragma unroll
            for (int w = 0; w < W; w++)
                if (B.active(w)) B.C(s, w) ^= P.R[w] ^ ((w == rs) ? (1ull << rl) : 0ull);
        }
        if (s == rs && lane == rl) {
#pragma unroll
            for (int w = 0; w < W; w++)
                if (B.active(w)) B.C(s, w) = P.R[w] | ((w == rs) ? (1ull << rl) : 0ull);
        }
    }
    bool sp_hit = false;
#pragma unroll
    for (int s = 0; s < W; s++)
        if (s == rs) {
            B.piv[s] |= 1ull << rl;
            sp_hit = (B.sp[s] >> rl) & 1ull;
        }
    if (lane == 0) S.colAt[rs * 64 + rl] = col;
    if (sp_hit) {
#pragma unroll
        for (int s = 0; s < W; s++) B.sp[s] ^= P.bp[s];
    }
#pragma unroll
    for (int s = 0; s < W; s++) {
        B.piv[s] = uniform64(B.piv[s]);
        B.sp[s] = uniform64(B.sp[s]);
    }
}

// The register basis reduces the column in the tier of the slices in use (a shot whose clusters
// hold at most 64 rows costs a one-slice reduction); the device-memory basis tests each slice at
// run time.
template <int W, class BB>
__device__ __forceinline__ bool insert_column(BB &B, const LsdLds &S, int col, int lane, int lr_src, int base, int cw) {
    InsertPlan<W> P;
    bool piv;
    if constexpr (!BB::kInMem && W == 2) {
        piv = B.ns <= 1 ? insert_plan<W, 1>(B, lane, lr_src, base, cw, P) : insert_plan<W, W>(B, lane, lr_src, base, cw, P);
    } else if constexpr (!BB::kInMem && W == 4) {
        piv = B.ns <= 1   ? insert_plan<W, 1>(B, lane, lr_src, base, cw, P)
              : B.ns <= 2 ? insert_plan<W, 2>(B, lane, lr_src, base, cw, P)
                          : insert_plan<W, W>(B, lane, lr_src, base, cw, P);
    } else if constexpr (BB::kInMem && W >= 8) {
        // memory bases: tiers of four slices (the loops still test each slice at run time)
        if (B.ns <= 4) piv = insert_plan<W, 4>(B, lane, lr_src, base, cw, P);
        else if (W > 8 && B.ns <= 8) piv = insert_plan<W, (W > 8 ? 8 : W)>(B, lane, lr_src, base, cw, P);
        else piv = insert_plan<W, W>(B, lane, lr_src, base, cw, P);
    } else {
        piv = insert_plan<W, W>(B, lane, lr_src, base, cw, P);
    }
    if (!piv) return false;
    insert_apply<W>(B, S, col, lane, P);
    return true;
}

__device__ __forceinline__ bool in_col(const uint32_t *incol, int j) { return (incol[j >> 5] >> (j & 31)) & 1u; }


// Local exhaustive reprocessing of order w (Appendix D) for every cluster that is not frozen.
// T = the cluster's dependent columns in ascending key, T_w its first w = min(mu, |T|).  Every
// pattern t over T_w fixes x_T = t and the pivot part x_P = x0 + sum_{k in t} z_k, where z_k is
// the pivot combination of column T_k (every T_k lies in the span of the pivots).  The cost is
// the integer weight of the set columns; the strictly smallest cost wins, the smaller t on ties.
// Patterns are spread over the lanes.
// Integer weight of the pivot columns set in x (uniform; every lane computes the same sum).
template <int W>
__device__ __forceinline__ int64_t pivot_cost(const LsdLds &S, const uint64_t (&x)[W]) {
    int64_t cost = 0;
#pragma unroll
    for (int s = 0; s < W; s++) {
        uint64_t v = x[s];
        while (v) {
            cost += S.wq[s * 64 + __builtin_ctzll(v)];
            v &= v - 1;
        }
    }
    return cost;
}

// z: the pivot rows of cluster c (inC) whose combination reproduces column col.
template <int W, class G, class BB>
__device__ __forceinline__ void column_combination(const LsdLds &S, const G &g, const BB &B, const uint64_t (&inC)[W],
                                                   int col, int lane, uint64_t (&z)[W]) {
    constexpr int K = 64 * W;
    uint32_t bf = 0;
    for (int e = g.col_ptr(col); e < g.col_ptr(col + 1); e++) {
        const int lr = S.loc[g.row_idx(e)];
        if (lr >= 0 && lr < K && (lr & 63) == lane) bf |= 1u << (lr >> 6);
    }
    uint64_t a[W];
#pragma unroll
    for (int s = 0; s < W; s++) a[s] = ballot((bf >> s) & 1u) & B.piv[s];
#pragma unroll
    for (int s = 0; s < W; s++) z[s] = ballot(((B.piv[s] & inC[s]) >> lane) & 1ull && parity_C<W>(B, s, a));
}

// Local OSD-CS (combination sweep) of one valid cluster c: candidates in the order zero pattern,
// every single dependent column of the cluster (T, ascending key), every pair (a, b), a < b < w,
// of its first w dependent columns (T_w, already selected into tsel/zk/tw); each scored by the
// integer weight of its solution; the strictly smallest cost wins, ties to the candidate met
// first.  xc: the cluster's LSD-0 solution over pivot rows.
template <int W, int KNP, class G, class BB>
__device__ void osd_cs_cluster(const LsdArgs &A, const LsdLds &S, const G &g, const BB &B, const uint64_t (&xc)[W],
                               const uint64_t (&inC)[W], int c, int nnp, int w, const float *llr, int lane) {
    const int64_t cost0 = pivot_cost<W>(S, xc);
    // singles: every dependent column of the cluster, best (cost, key)
    int64_t bs_cost = INT64_MAX;
    uint64_t bs_key = ~0ull;
    for (int e = 0; e < nnp; e++) {
        const int col = __builtin_amdgcn_readfirstlane(S.colNP[e]);
        const int rr = S.loc[g.row_idx(g.col_ptr(col))];
        if (__builtin_amdgcn_readfirstlane(S.croot[rr]) != c) continue;
        uint64_t z[W], x[W];
        column_combination<W>(S, g, B, inC, col, lane, z);
#pragma unroll
        for (int s = 0; s < W; s++) x[s] = xc[s] ^ z[s];
        const int64_t cost = pivot_cost<W>(S, x) + A.omega[col];
        const uint32_t kj = (G::kInLds || A.keys_in_lds) ? S.keys[col] : ordered_key(llr[col]);
        const uint64_t key = ((uint64_t)kj << 32) | (uint32_t)col;
        if (cost < bs_cost || (cost == bs_cost && key < bs_key)) { bs_cost = cost; bs_key = key; }
    }
    // pairs among T_w, lexicographic index order
    const int npair = w * (w - 1) / 2;
    uint64_t bp = ~0ull;  // (cost + 2^50) << 12 | pair index, the smallest per lane
    for (int p = lane; p < npair; p += 64) {
        int a = 0, rem = p;
        while (rem >= w - 1 - a) { rem -= w - 1 - a; a++; }
        const int b = a + 1 + rem;
        uint64_t x[W];
#pragma unroll
        for (int s = 0; s < W; s++) x[s] = xc[s] ^ S.zk[a * W + s] ^ S.zk[b * W + s];
        const int64_t cost = pivot_cost<W>(S, x) + S.tw[a] + S.tw[b];
        const uint64_t key = ((uint64_t)(cost + (1ll << 50)) << 12) | (uint64_t)p;
        bp = key < bp ? key : bp;
    }
    bp = wave_min_u64(bp);
    const int64_t bp_cost = bp == ~0ull ? INT64_MAX : (int64_t)(bp >> 12) - (1ll << 50);
    uint64_t x[W];
#pragma unroll
    for (int s = 0; s < W; s++) x[s] = xc[s];
    if (bs_cost < cost0 && bs_cost <= bp_cost) {
        const int col = (int)(uint32_t)bs_key;
        uint64_t z[W];
        column_combination<W>(S, g, B, inC, col, lane, z);
#pragma unroll
        for (int s = 0; s < W; s++) x[s] ^= z[s];
        if (lane == 0) atomicOr(&S.cbit[col >> 5], 1u << (col & 31));
    } else if (bp_cost < cost0 && bp_cost < bs_cost) {
        const int p = (int)(bp & 4095ull);
        int a = 0, rem = p;
        while (rem >= w - 1 - a) { rem -= w - 1 - a; a++; }
        const int b = a + 1 + rem;
#pragma unroll
        for (int s = 0; s < W; s++) x[s] ^= S.zk[a * W + s] ^ S.zk[b * W + s];
        if (lane == 0) {
            atomicOr(&S.cbit[S.tsel[a] >> 5], 1u << (S.tsel[a] & 31));
            atomicOr(&S.cbit[S.tsel[b] >> 5], 1u << (S.tsel[b] & 31));
        }
    }
#pragma unroll
    for (int s = 0; s < W; s++)
        if ((x[s] >> lane) & 1ull) {
            const int col = S.colAt[s * 64 + lane];
            atomicOr(&S.cbit[col >> 5], 1u << (col & 31));
        }
    wave_sync();
}

// KNP: capacity of the dependent-column list colNP (at most 64 * 64 entries).
template <int W, int KNP, class G, class BB>
__device__ void osd_e_clusters(const LsdArgs &A, const LsdLds &S, const G &g, const BB &B,
                               const uint64_t (&x0)[W], int nrows, int npc, const float *llr, int lane) {
    constexpr int K = 64 * W;
    // OSD-E: T_w = the first min(mu, |T|) columns; OSD-CS: pairs among the first min(w, |T|)
    const int mu = A.cs_order > 0 ? (A.cs_order < kMaxMu ? A.cs_order : kMaxMu) : (A.mu < kMaxMu ? A.mu : kMaxMu);
#pragma unroll
    for (int s = 0; s < W; s++) {
        const int r = s * 64 + lane;
        if ((B.piv[s] >> lane) & 1ull) S.wq[r] = A.omega[S.colAt[r]];
    }
    uint64_t roots[W];
#pragma unroll
    for (int s = 0; s < W; s++) {
        const int r = s * 64 + lane;
        roots[s] = ballot(r < nrows && S.croot[r] == r && S.state[r] != kFrozen);
    }
    wave_sync();
    const int nnp = npc < KNP ? npc : KNP;
    using Chosen = typename std::conditional<(KNP > 32 * 64), uint64_t, uint32_t>::type;
#pragma unroll
    for (int s0 = 0; s0 < W; s0++) {
        while (roots[s0]) {
            const int c = s0 * 64 + __builtin_ctzll(roots[s0]);
            roots[s0] &= roots[s0] - 1;
            uint64_t inC[W];
#pragma unroll
            for (int s = 0; s < W; s++) {
                const int r = s * 64 + lane;
                inC[s] = ballot(r < nrows && S.croot[r] == c);
            }
            // T_w: the cluster's dependent columns of smallest key
            Chosen chosen = 0;  // bit u: entry lane + 64 u taken
            int w = 0;
            for (; w < mu; w++) {
                uint64_t mine = ~0ull;
                for (int u = 0; u * 64 + lane < nnp; u++) {
                    if ((chosen >> u) & Chosen(1)) continue;
                    const int col = S.colNP[u * 64 + lane];
                    const int rr = S.loc[g.row_idx(g.col_ptr(col))];
                    if (S.croot[rr] != c) continue;
                    const uint32_t kj = (G::kInLds || A.keys_in_lds) ? S.keys[col] : ordered_key(llr[col]);
                    const uint64_t key = ((uint64_t)kj << 32) | (uint32_t)col;
                    mine = key < mine ? key : mine;
                }
                const uint64_t kmin = wave_min_u64(mine);
                if (kmin == ~0ull) break;
                const int col = (int)(uint32_t)kmin;
                for (int u = 0; u * 64 + lane < nnp; u++)
                    if (S.colNP[u * 64 + lane] == col) chosen |= Chosen(1) << u;
                // z_w: pivot rows of this cluster whose combination reproduces column col
                uint32_t bf = 0;
                for (int e = g.col_ptr(col); e < g.col_ptr(col + 1); e++) {
                    const int lr = S.loc[g.row_idx(e)];
                    if (lr >= 0 && lr < K && (lr & 63) == lane) bf |= 1u << (lr >> 6);
                }
                uint64_t a[W];
#pragma unroll
                for (int s = 0; s < W; s++) a[s] = ballot((bf >> s) & 1u) & B.piv[s];
#pragma unroll
                for (int s = 0; s < W; s++) {
                    const uint64_t z = ballot(((B.piv[s] & inC[s]) >> lane) & 1ull && parity_C<W>(B, s, a));
                    if (lane == 0) S.zk[w * W + s] = z;
                }
                if (lane == 0) {
                    S.tsel[w] = col;
                    S.tw[w] = A.omega[col];
                }
            }
            wave_sync();
            uint64_t xc[W];
#pragma unroll
            for (int s = 0; s < W; s++) xc[s] = x0[s] & inC[s];
            if (A.cs_order > 0) {
                osd_cs_cluster<W, KNP>(A, S, g, B, xc, inC, c, nnp, w, llr, lane);
                continue;
            }
            // search the 2^w patterns
            const int npat = 1 << w;
            uint64_t best = ~0ull;
            for (int pt = lane; pt < npat; pt += 64) {
                uint64_t x[W];
                int64_t cost = 0;
#pragma unroll
                for (int s = 0; s < W; s++) x[s] = xc[s];
                for (int k = 0; k < w; k++) {
                    if ((pt >> k) & 1) {
                        cost += S.tw[k];
#pragma unroll
                        for (int s = 0; s < W; s++) x[s] ^= S.zk[k * W + s];
                    }
                }
#pragma unroll
                for (int s = 0; s < W; s++) {
                    uint64_t v = x[s];
                    while (v) {
                        cost += S.wq[s * 64 + __builtin_ctzll(v)];
                        v &= v - 1;
                    }
                }
                const uint64_t key = ((uint64_t)(cost + (1ll << 50)) << 12) | (uint64_t)pt;
                best = key < best ? key : best;
            }
            const int tb = (int)(wave_min_u64(best) & 4095ull);
            uint64_t x[W];
#pragma unroll
            for (int s = 0; s < W; s++) x[s] = xc[s];
            for (int k = 0; k < w; k++) {
                if ((tb >> k) & 1) {
#pragma unroll
                    for (int s = 0; s < W; s++) x[s] ^= S.zk[k * W + s];
                    if (lane == 0) atomicOr(&S.cbit[S.tsel[k] >> 5], 1u << (S.tsel[k] & 31));
                }
            }
#pragma unroll
            for (int s = 0; s < W; s++)
                if ((x[s] >> lane) & 1ull) {
                    const int col = S.colAt[s * 64 + lane];
                    atomicOr(&S.cbit[col >> 5], 1u << (col & 31));
                }
            wave_sync();
        }
    }
}

// One batch of the round's new columns reduced together (insert_round_batched): `mark` tags the
// local rows of the batch's columns in lroot, the cluster slots are in selu (per root: its pivot
// row, then the lane of its batch column), and `stage` receives the new pivot rows' Mrow words.
// NS as for insert_plan.  dep: this lane's column (inb) turned out dependent.
template <int W, int NS, class BB>
__device__ __forceinline__ void reduce_batch(BB &B, const LsdLds &S, int lane, int mark, bool inb, int root, int col,
                                             const int (&crv)[W], bool &dep) {
    uint32_t *selu = (uint32_t *)S.sel;
    uint64_t *stage = S.lkey;
    uint32_t bf = 0;  // bit s: local row 64 s + lane lies in its cluster's batch column
#pragma unroll
    for (int s = 0; s < NS; s++) bf |= (uint32_t)(S.lroot[s * 64 + lane] == mark) << s;
    uint64_t a[W];    // the batch columns' support on pivot rows
#pragma unroll
    for (int s = 0; s < W; s++) a[s] = s < NS ? ballot((bf >> s) & 1u) & B.piv[s] : 0ull;
    // a row's Mrow (and a pivot's CT) has bits only at its own cluster's pivots, so one parity
    // pass reduces every cluster's column on that cluster's rows
    uint32_t bpf = 0, cfl = 0;
#pragma unroll
    for (int s = 0; s < NS; s++) {
        if (!B.active(s)) continue;
        bpf |= (uint32_t)(((bf >> s) & 1u) ^ parity_M<W, BB, NS>(B, s, a)) << s;
        if (((B.piv[s] >> lane) & 1ull) && parity_C<W, BB, NS>(B, s, a)) cfl |= 1u << s;
    }
    // each cluster's pivot: its smallest local row in the reduced column (as a one-column
    // insertion picks it)
#pragma unroll
    for (int s = 0; s < NS; s++)
        if ((bpf >> s) & 1u) atomicMin(&selu[2 * crv[s]], (uint32_t)(s * 64 + lane));
    wave_sync();
    int pr[W], slot[W];
#pragma unroll
    for (int s = 0; s < W; s++) { pr[s] = -1; slot[s] = 0; }
#pragma unroll
    for (int s = 0; s < NS; s++) {
        if (((bpf | cfl) >> s) & 1u) {
            // a cluster whose column turned out dependent has no pivot (all ones): pr stays -1
            const uint32_t prv = selu[2 * crv[s]];
            pr[s] = prv < (uint32_t)(64 * W) ? (int)prv : -1;
            slot[s] = (int)(selu[2 * crv[s] + 1] & 63u);
            if (pr[s] == s * 64 + lane) {
#pragma unroll
                for (int w = 0; w < NS; w++) stage[slot[s] * W + w] = B.M(s, w);
            }
        }
    }
    dep = inb && selu[2 * root] == 0xffffffffu;  // no row of the cluster in the reduced column
    wave_sync();
    uint64_t newp[W], flip[W];
#pragma unroll
    for (int s = 0; s < NS; s++) {
        // rows of a cluster without a new pivot are left alone (a dependent column changes nothing)
        const bool rowb = ((bpf >> s) & 1u) && pr[s] >= 0, rowc = ((cfl >> s) & 1u) && pr[s] >= 0;
        const bool is_new = pr[s] == s * 64 + lane;
        bool sp_hit = false;
        if (rowb || rowc) {
            const int ps = pr[s] >> 6, pl = pr[s] & 63;
            uint64_t R[W];
#pragma unroll
            for (int w = 0; w < NS; w++) R[w] = stage[slot[s] * W + w];
            if (rowb) {
#pragma unroll
                for (int w = 0; w < NS; w++)
                    if (B.active(w)) B.M(s, w) ^= R[w] ^ ((w == ps) ? (1ull << pl) : 0ull);
            }
            if (rowc) {
#pragma unroll
                for (int w = 0; w < NS; w++)
                    if (B.active(w)) B.C(s, w) ^= R[w] ^ ((w == ps) ? (1ull << pl) : 0ull);
            }
            if (is_new) {
#pragma unroll
                for (int w = 0; w < NS; w++)
                    if (B.active(w)) B.C(s, w) = R[w] | ((w == ps) ? (1ull << pl) : 0ull);
            }
#pragma unroll
            for (int t = 0; t < NS; t++)
                if (t == ps) sp_hit = (B.sp[t] >> pl) & 1ull;
        }
        newp[s] = ballot(is_new);
        // the reduced syndrome changes by the reduced column wherever the cluster's pivot row
        // carries a syndrome bit
        flip[s] = ballot(rowb && sp_hit);
    }
    // the new pivots' columns: the pivot lane takes its cluster's batch column
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const int c = __shfl(col, slot[s], 64);
        if (pr[s] == s * 64 + lane) S.colAt[s * 64 + lane] = c;
    }
#pragma unroll
    for (int s = 0; s < NS; s++) {
        B.piv[s] = uniform64(B.piv[s] | newp[s]);
        B.sp[s] = uniform64(B.sp[s] ^ flip[s]);
    }
}

// Phase (4) with the cluster-batched schedule (rounds of kBatchMin to 64 selections): the round's
// distinct columns are grouped by the cluster they end up in after this round's merges, batch b
// holding every cluster's b-th column in ascending key, so a batch has at most one column per
// cluster.  Clusters own disjoint local rows, so a batch is reduced in one pass (reduce_batch) with
// the same pivots and the same dependent columns as inserting its columns one by one in key order
// -- the paper's parallelism across clusters, spread over the lanes of the shot's wavefront.
// lkey is read into registers first (it then serves as the staging area); the cluster slots in
// the selection array are all ones again on return, and the marks in lroot are never read back.
template <int W, bool MU, int KNP, class G, class BB>
__device__ __forceinline__ void insert_round_batched(const LsdArgs &A, const LsdLds &S, const G &g, BB &B, int nsel,
                                                     int rounds, int &npc, int lane) {
    const bool selp = lane < nsel;
    const uint64_t kp = selp ? S.lkey[lane] : ~0ull;
    const int col = (int)(uint32_t)kp;
    int root = 0;
    if (selp) root = S.croot[S.loc[g.row_idx(g.col_ptr(col))]];  // every row points at its root here
    int crv[W];
#pragma unroll
    for (int s = 0; s < W; s++) crv[s] = S.croot[s * 64 + lane];
    bool dup = !selp;
    for (int q = 0; q < nsel; q++) dup |= readlane64(kp, q) == kp && q < lane;
    int bidx = 0;  // distinct columns of the same cluster with a smaller key
    for (int q = 0; q < nsel; q++) {
        const bool dq = __builtin_amdgcn_readlane((int)dup, q) != 0;
        bidx += (!dq && __builtin_amdgcn_readlane(root, q) == root && readlane64(kp, q) < kp) ? 1 : 0;
    }
    uint32_t *selu = (uint32_t *)S.sel;
    wave_sync();  // every lane has read lkey before it becomes the staging area
    for (int b = 0;; b++) {
        const bool inb = !dup && bidx == b;
        if (!ballot(inb)) break;
        const int mark = -2 - b - 64 * rounds;  // below -1: no root, stamp or earlier mark of the shot
        if (inb) {
            const int c0 = g.col_ptr(col), c1 = g.col_ptr(col + 1);
            for (int e = c0; e < c1; e++) {
                const int lr = S.loc[g.row_idx(e)];
                S.lroot[lr] = mark;
                S.cand[lr] = kStale;
            }
            atomicOr(&S.incol[col >> 5], 1u << (col & 31));
            selu[2 * root + 1] = (uint32_t)lane;
        }
        wave_sync();
        bool dep = false;
        if constexpr (BB::kInMem) {
            reduce_batch<W, W>(B, S, lane, mark, inb, root, col, crv, dep);
        } else {
            if (B.ns <= 1) reduce_batch<W, 1>(B, S, lane, mark, inb, root, col, crv, dep);
            else if (B.ns <= 2) reduce_batch<W, (W < 2 ? W : 2)>(B, S, lane, mark, inb, root, col, crv, dep);
            else reduce_batch<W, W>(B, S, lane, mark, inb, root, col, crv, dep);
        }
        if constexpr (MU) {
            if (A.mu > 0) {
                const uint64_t dball = ballot(dep);
                if (dep) {
                    const int at = npc + __popcll(dball & ((1ull << lane) - 1ull));
                    if (at < KNP) S.colNP[at] = col;
                }
                npc += __popcll(dball);
            }
        }
        wave_sync();
        if (inb) {  // the cluster slots back to all ones for the next batch and the next round
            selu[2 * root] = 0xffffffffu;
            selu[2 * root + 1] = 0xffffffffu;
        }
        wave_sync();
    }
}

// MU: the decoder runs LSD-mu (A.mu > 0); decoders without it get no LSD-mu code at all, which
// leaves the register allocator more room in the LSD-0 rounds.
// WIDE: the basis lives in memory at basis_mem (this wavefront's [2][W][W][64] words: in LDS when
// BLDS, else in device memory) and
// only the slices of local rows in use are visited; the other kernels keep it in registers.
// OVF: a shot that outgrows the capacity is appended to A.ovf_list (when set) for the next
// overflow kernel.
// CB: the cluster-batched schedule of phase (4) (insert_round_batched); same results.
template <int W, bool MU, class G, bool WIDE = false, bool OVF = false, bool BLDS = false, bool CB = false>
__device__ __forceinline__ void decode_shot(const LsdArgs &A, const LsdLds &S, const G &g, int shot, int lane,
                            uint64_t *basis_mem = nullptr) {
    constexpr int K = 64 * W;
    constexpr int KNP = WIDE ? kWideDependent : K;  // capacity of the dependent-column list
    const int m = A.g.m, n = A.g.n;
    const float *llr = A.llr + (size_t)shot * n;
    const uint8_t *syn = A.syn + (size_t)shot * m;
    uint8_t *corr = A.corr + (size_t)shot * n;

    // the syndrome of the first detectors is loaded together with the LLRs (one memory round trip
    // before the seeds; the rest, if m > 256, is read where it is used)
    constexpr int kSynPre = W < 4 ? W : 4;  // chunks of 64 detectors (m <= 64 W for W < 4)
    uint8_t sy[kSynPre];
#pragma unroll
    for (int q = 0; q < kSynPre; q++) sy[q] = q * 64 + lane < m ? syn[q * 64 + lane] : 0;
    bool nan = false;
    for (int j = lane; j < n; j += 64) {
        // coherent read: an equal compare-and-swap returns the word at the point of coherence
        const float v = A.coherent_llr ? __int_as_float(atomicCAS((int *)llr + j, 0, 0)) : llr[j];
        nan |= (v != v);
        if (G::kInLds || A.keys_in_lds) S.keys[j] = ordered_key(v);
    }
    for (int w = lane; w < (n + 31) / 32; w += 64) { S.incol[w] = 0u; S.cbit[w] = 0u; }
    for (int i = lane; i < m; i += 64) { S.loc[i] = -1; S.claimer[i] = kFree; }
    for (int r = lane; r < K; r += 64) {
        S.lroot[r] = -1;    // validity stamps of an earlier shot
        S.sel[r] = ~0ull;   // per-root selection (cleared again as each round reads it)
    }
    wave_sync();

    // the correction row from the bit vector, written once on every exit
    auto write_row = [&]() {
        wave_sync();
        if ((n & 15) == 0 && (((uintptr_t)corr) & 15) == 0) {
            for (int c = lane; c < (n >> 4); c += 64) {
                const uint32_t bits = (S.cbit[c >> 1] >> ((c & 1) * 16)) & 0xffffu;
                uint32_t v[4];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const uint32_t nb = bits >> (4 * k);
                    v[k] = (nb & 1u) | ((nb & 2u) << 7) | ((nb & 4u) << 14) | ((nb & 8u) << 21);
                }
                ((uint4 *)corr)[c] = make_uint4(v[0], v[1], v[2], v[3]);
            }
        } else {
            for (int j = lane; j < n; j += 64) corr[j] = (uint8_t)((S.cbit[j >> 5] >> (j & 31)) & 1u);
        }
    };

    uint8_t status = QLSD_ST_LSD_RUN;
    int rounds = 0;
    auto finish = [&](uint8_t st, int ncl, int maxc) {
        if (A.cstats && ncl == 0 && lane == 0) A.cstats[shot] = qlsd_cluster_stats{0, 0, 0, 0};
        if (A.info && lane == 0) {
            qlsd_shot_info inf;
            inf.status = st;
            inf.reserved = 0;
            inf.bp_iters = (int16_t)A.bp_iters;
            inf.n_clusters = (int16_t)ncl;
            inf.rounds = (int16_t)rounds;
            inf.max_cluster_cols = maxc;
            A.info[shot] = inf;
        }
    };
    if (ballot(nan)) {
        write_row();
        finish(QLSD_ST_LSD_RUN | QLSD_ST_BAD_LLR, 0, 0);
        return;
    }
    // capacity exceeded: the shot reports OVERFLOW with a zero correction (the bit vector is
    // only filled by the solve, after the last capacity check)
    auto overflow = [&](uint8_t st) {
        write_row();
        finish(st | QLSD_ST_OVERFLOW, 0, 0);
        // hand the shot to the next overflow kernel (launched after this one), which rewrites both
        if constexpr (OVF) {
            if (A.ovf_list && lane == 0) A.ovf_list[atomicAdd(A.ovf_count, 1)] = shot;
        }
    };

    // clusters: one per flipped detector, local rows in ascending detector order
    int nrows = 0;
    for (int i0 = 0; i0 < m; i0 += 64) {
        const int i = i0 + lane;
        uint8_t sv = 0;
#pragma unroll
        for (int q = 0; q < kSynPre; q++)
            if (i0 == q * 64) sv = sy[q];
        if (i0 >= kSynPre * 64 && i < m) sv = syn[i];
        const bool f = i < m && (sv & 1);
        const uint64_t bal = ballot(f);
        if (f) {
            const int idx = nrows + __popcll(bal & ((1ull << lane) - 1ull));
            if (idx < K) {
                S.loc[i] = idx;
                S.rowOf[idx] = i;
                S.croot[idx] = idx;
                S.state[idx] = kInvalid;
                S.cand[idx] = kStale;
            }
        }
        nrows += __popcll(bal);
    }
    if (nrows == 0) {
        write_row();
        finish(QLSD_ST_LSD_RUN, 0, 0);
        return;
    }
    if (nrows > K) { overflow(QLSD_ST_LSD_RUN); return; }
    const int nseed = nrows;
    if (lane == 0) S.ctl[0] = nrows;

    Basis<W, WIDE, BLDS> B;
    if constexpr (WIDE) {
        // rows and pivots only ever occupy the first min(ceil(m/64), W) slices (a shot with more
        // rows has overflowed); the rest stays untouched
        B.mem = (typename Basis<W, true, BLDS>::Ptr)basis_mem + lane;
        const int msl = min((m + 63) >> 6, W);
        for (int s = 0; s < msl; s++)
            for (int w = 0; w < msl; w++) { B.M(s, w) = 0; B.C(s, w) = 0; }
    }
    B.ns = (nrows + 63) >> 6;
#pragma unroll
    for (int s = 0; s < W; s++) {
        if constexpr (!WIDE) {
#pragma unroll
            for (int w = 0; w < W; w++) { B.M(s, w) = 0; B.C(s, w) = 0; }
        }
        B.piv[s] = 0;
        const int lo = s * 64;
        B.sp[s] = nseed >= lo + 64 ? ~0ull : (nseed > lo ? ((1ull << (nseed - lo)) - 1ull) : 0ull);
    }
    wave_sync();

    // LSD-0 rounds grow the invalid clusters until none is left; LSD-mu then runs mu more
    // rounds in which every cluster that is not frozen grows (Appendix D).
    bool grow_all = false;
    int mu_left = 0;
    int npc = 0;  // dependent columns recorded in colNP
    for (;;) {
        // (1) selection: per growing root, the candidate of smallest key (round-start state);
        // every entry of sel is ~0 here
        // Branch-light: a row's root and cached candidate are read together, then the root's
        // state (reads of rows past nrows are in bounds and unused); a row rescans only when
        // marked kStale.
#pragma unroll
        for (int s = 0; s < W; s++) {
            if (s * 64 >= nrows) break;
            const int r = s * 64 + lane;
            const bool valid = r < nrows;
            const int cr = S.croot[r];
            uint64_t best = S.cand[r];
            // a graph in LDS: the row's edge range is read alongside (rows past nrows hold a stale
            // detector of an earlier shot, or nothing yet: clamped to a valid index)
            int e0 = 0, e1 = 0;
            if constexpr (G::kInLds) {
                const int d = S.rowOf[r];
                const int dd = (unsigned)d < (unsigned)m ? d : 0;
                e0 = g.row_ptr(dd);
                e1 = g.row_ptr(dd + 1);
            }
            const int c = valid ? cr : 0;
            const uint8_t st = S.state[c];
            const bool grow = valid && ((MU && grow_all) ? st != kFrozen : st == kInvalid);
            {
                {
                    if (grow && best == kStale) {
                        best = ~0ull;
                        if constexpr (!G::kInLds) {
                            const int d = S.rowOf[r];
                            e0 = g.row_ptr(d);
                            e1 = g.row_ptr(d + 1);
                        }
                        // kScan entries per pass, every load issued before any is used (entries
                        // past the row's end re-read its last one and are masked out), so a row of
                        // weight <= kScan costs two dependent rounds of loads (6 fits the small
                        // codes' rows without masked slots; the large graphs' rows are longer)
                        constexpr int kScan = W <= 2 ? 6 : 8;
                        for (int eb = e0; eb < e1; eb += kScan) {
                            int jj[kScan];
#pragma unroll
                            for (int u = 0; u < kScan; u++) jj[u] = g.col_idx(min(eb + u, e1 - 1));
                            uint32_t kk[kScan], ic[kScan];
#pragma unroll
                            for (int u = 0; u < kScan; u++) {
                                kk[u] = (G::kInLds || A.keys_in_lds) ? S.keys[jj[u]] : ordered_key(llr[jj[u]]);
                                ic[u] = S.incol[jj[u] >> 5];
                            }
#pragma unroll
                            for (int u = 0; u < kScan; u++) {
                                const bool ok = eb + u < e1 && !((ic[u] >> (jj[u] & 31)) & 1u);
                                const uint64_t key = ok ? (((uint64_t)kk[u] << 32) | (uint32_t)jj[u]) : ~0ull;
                                best = key < best ? key : best;
                            }
                        }
                        S.cand[r] = best;
                    }
                    if (grow && best != ~0ull) atomicMin((unsigned long long *)&S.sel[c], (unsigned long long)best);
                }
            }
        }
        wave_sync();
        // (2) compact list of (root, key); an invalid root with no candidate is frozen (UNSAT)
        int nsel = 0;
#pragma unroll
        for (int s = 0; s < W; s++) {
            if (s * 64 >= nrows) break;
            const int r = s * 64 + lane;
            const int cr = S.croot[r];
            const uint8_t st = S.state[r];
            const uint64_t key = S.sel[r];
            if (key != ~0ull) S.sel[r] = ~0ull;  // ready for the next round
            const bool growing = r < nrows && cr == r && ((MU && grow_all) ? st != kFrozen : st == kInvalid);
            const bool take = growing && key != ~0ull;
            if (growing && key == ~0ull && st == kInvalid) {
                S.state[r] = kFrozen;
                status |= QLSD_ST_UNSAT;
            }
            const uint64_t bal = ballot(take);
            if (take) {
                const int p = nsel + __popcll(bal & ((1ull << lane) - 1ull));
                S.lkey[p] = key;
                S.lroot[p] = r;
            }
            nsel += __popcll(bal);
        }
        if (ballot(status & QLSD_ST_UNSAT)) status |= QLSD_ST_UNSAT;
        wave_sync();
        if (nsel == 0) {
            if (MU && !grow_all && A.mu > 0) {  // every invalid cluster is frozen; valid ones may still grow
                grow_all = true;
                mu_left = A.mu;
                continue;
            }
            break;
        }

        // (3) claims and unions (Def. 4.4): pairs (selection, detector of its fault)
        const int cwm = g.max_cw;
        const int npairs = nsel * cwm;
        // pair id -> (selection, entry): id / cwm as a multiply-high by ceil(2^32 / cwm), exact for
        // id < 2^16 and cwm <= 16
        const uint64_t cw_magic = (0x100000000ull + (uint64_t)cwm - 1ull) / (uint64_t)cwm;  // 2^32 when cwm = 1
        // pair id -> (detector d, claiming root c); false for padding entries of short columns
        auto pair_of = [&](int id, int &d, int &c) -> bool {
            const int p = (int)(((uint64_t)(uint32_t)id * cw_magic) >> 32), u = id - p * cwm;
            const int col = (int)(uint32_t)S.lkey[p];
            const int c0 = g.col_ptr(col), c1 = g.col_ptr(col + 1);
            c = S.lroot[p];
            const bool ok = u < c1 - c0;
            d = g.row_idx(ok ? c0 + u : c0);  // a picked fault has at least one detector
            return ok;
        };
        // this lane's first pair is decoded once and kept for the unions
        int d0 = 0, c0p = 0, loc0 = -1;
        const bool has0 = lane < npairs && pair_of(lane, d0, c0p);
        if (has0) {
            loc0 = S.loc[d0];
            if (loc0 < 0) atomicMin(&S.claimer[d0], c0p);
        }
        for (int id = lane + 64; id < npairs; id += 64) {
            int d, c;
            if (pair_of(id, d, c) && S.loc[d] < 0) atomicMin(&S.claimer[d], c);
        }
        wave_sync();
        bool merged = false;
        auto join = [&](int d, int c) {
            const int cl = S.claimer[d];
            if (cl != kFree) {
                if (cl == c) {
                    const int idx = atomicAdd(&S.ctl[0], 1);
                    if (idx < K) {
                        S.rowOf[idx] = d;
                        S.croot[idx] = c;
                        S.state[idx] = kValid;
                        S.cand[idx] = kStale;
                        S.loc[d] = idx;
                    }
                } else {
                    merged |= unite(S.croot, c, cl);
                }
            } else {
                merged |= unite(S.croot, c, S.croot[S.loc[d]]);
            }
        };
        int nrows_new;
        if (npairs <= 64) {
            // one pair per lane: the claimed detectors become local rows nrows, nrows + 1, ... in
            // lane order (any numbering of the new rows gives the same pivot columns and solution)
            // detectors clustered before the round were never claimed
            const int cl = has0 && loc0 < 0 ? S.claimer[d0] : kFree;
            const bool add = has0 && cl != kFree && cl == c0p;
            const uint64_t bal = ballot(add);
            if (add) {
                const int idx = nrows + __popcll(bal & ((1ull << lane) - 1ull));
                if (idx < K) {
                    S.rowOf[idx] = d0;
                    S.croot[idx] = c0p;
                    S.state[idx] = kValid;
                    S.cand[idx] = kStale;
                    S.loc[d0] = idx;
                }
            } else if (has0) {
                // claimed by a smaller root, or clustered before the round: in the common case the
                // detector is the picking cluster's own (its row points at that round-start root)
                int other = cl;
                if (cl == kFree) other = S.croot[loc0];
                if (other != c0p) merged |= unite(S.croot, c0p, other);
            }
            nrows_new = nrows + __popcll(bal);
            if (lane == 0) S.ctl[0] = nrows_new;
        } else {
            if (has0) join(d0, c0p);
            for (int id = lane + 64; id < npairs; id += 64) {
                int d, c;
                if (pair_of(id, d, c)) join(d, c);
            }
        }
        const bool any_merge = ballot(merged) != 0ull;
        wave_sync();
        if (npairs > 64) nrows_new = __builtin_amdgcn_readfirstlane(S.ctl[0]);
        if (nrows_new > K) { overflow(status); return; }
        // flatten the forest (only after a merge: otherwise every row already points at a root,
        // new rows at the round-start root that claimed them); release this round's claims
        if (any_merge) {
#pragma unroll
            for (int s = 0; s < W; s++) {
                const int r = s * 64 + lane;
                if (r < nrows_new) S.croot[r] = find_root(S.croot, r);
            }
        }
        // release this round's claims: with at most 64 pairs each pair's lane holds its detector
        // (detectors clustered before the round were never claimed: writing kFree is a no-op)
        if (npairs <= 64) {
            if (has0) S.claimer[d0] = kFree;
        } else {
            for (int r = nrows + lane; r < nrows_new; r += 64) S.claimer[S.rowOf[r]] = kFree;
        }
        nrows = nrows_new;
        B.ns = (nrows + 63) >> 6;
        wave_sync();

        // (4) the round's distinct new columns, ascending key, each reduced on the fly.  Order:
        // entry p goes to position rank(p) = number of entries with a smaller key (distinct keys get
        // distinct positions; a column picked by several clusters is placed once, by its first
        // entry).  The selection array is free at this point and holds the order.
        // With at most 64 (selection, entry) pairs (the usual case) the ranks stay in registers
        // (lane p: selection p) and each pair's local row is read once, here, for all columns of the
        // round at the same time (lane id: pair id, as in the claims); otherwise an order array in
        // LDS and per-column lookups.
        bool batched = false;
        if constexpr (CB) {
            // the cluster-batched schedule: several clusters growing at once have their columns
            // reduced together
            if (nsel >= kBatchMin && nsel <= 64) {
                insert_round_batched<W, MU, KNP>(A, S, g, B, nsel, rounds, npc, lane);
                batched = true;
            }
        }
        if (!batched) {
            const bool fast = npairs <= 64;
            int32_t *order = (int32_t *)S.sel;
            int rank = 0, colp = 0, lr_pair = -1;
            bool dup = true;
            if (fast) {
                const uint64_t kp = lane < nsel ? S.lkey[lane] : ~0ull;
                lr_pair = has0 ? S.loc[d0] : -1;
                bool seen = false;
                for (int q = 0; q < nsel; q++) {
                    const uint64_t kq = readlane64(kp, q);
                    rank += kq < kp ? 1 : 0;
                    seen |= kq == kp && q < lane;
                }
                dup = lane >= nsel || seen;
                colp = (int)(uint32_t)kp;
            } else {
                for (int p = lane; p < nsel; p += 64) order[p] = -1;
                wave_sync();
                for (int p = lane; p < nsel; p += 64) {
                    const uint64_t kp = S.lkey[p];
                    int rk = 0;
                    bool dp = false;
                    for (int q = 0; q < nsel; q++) {
                        const uint64_t kq = S.lkey[q];
                        rk += kq < kp ? 1 : 0;
                        dp |= kq == kp && q < p;
                    }
                    if (!dp) order[rk] = (int)(uint32_t)kp;
                }
                wave_sync();
            }
            for (int r = 0; r < nsel; r++) {
                int col, lr_src, base, cwc;
                if (fast) {
                    const uint64_t at = ballot(!dup && rank == r);
                    if (!at) continue;
                    const int p = __builtin_ctzll(at);
                    col = __builtin_amdgcn_readlane(colp, p);
                    lr_src = lr_pair;
                    base = p * cwm;
                    cwc = cwm;
                } else {
                    col = order[r];
                    if (col < 0) continue;
                    const int c0 = g.col_ptr(col);
                    cwc = g.col_ptr(col + 1) - c0;
                    lr_src = lane < cwc ? S.loc[g.row_idx(c0 + lane)] : -1;
                    base = 0;
                }
                // wave-uniform: lets the entry loop in insert_column run on scalar registers
                col = __builtin_amdgcn_readfirstlane(col);
                base = __builtin_amdgcn_readfirstlane(base);
                cwc = __builtin_amdgcn_readfirstlane(cwc);
                // no read of incol or cand before the next sync: the updates need not return
                if (lane == 0) atomicOr(&S.incol[col >> 5], 1u << (col & 31));
                if (lane >= base && lane < base + cwc && lr_src >= 0) S.cand[lr_src] = kStale;
                const bool pivot = insert_column<W>(B, S, col, lane, lr_src, base, cwc);
                if (MU && !pivot && A.mu > 0) {
                    if (lane == 0 && npc < KNP) S.colNP[npc] = col;
                    npc++;
                }
            }
            // the order array lives in the selection array, which the next round needs cleared
            if (!fast)
                for (int p = lane; p < (nsel + 1) / 2; p += 64) S.sel[p] = ~0ull;
        }
        wave_sync();

        // (5) validity: a cluster is valid iff its reduced syndrome vanishes.  Every row points at
        // its root here.  Each row that keeps a reduced-syndrome bit stamps its root's entry of
        // the selection-root array (free at this point) with K + rounds, which no entry written
        // this shot holds otherwise (the array is cleared per shot and else holds roots < K);
        // after a sync each root reads its own entry, and the states are written once.
        int32_t *vmark = S.lroot;
        const int stamp = K + rounds;
        int crv[W];
        uint8_t stv[W];
#pragma unroll
        for (int s = 0; s < W; s++) {
            const int r = s * 64 + lane;
            crv[s] = S.croot[r];
            stv[s] = S.state[r];
            if (r < nrows && ((B.sp[s] >> lane) & 1ull)) vmark[crv[s]] = stamp;
        }
        wave_sync();
        bool inv_mine = false;
#pragma unroll
        for (int s = 0; s < W; s++) {
            const int r = s * 64 + lane;
            if (r < nrows && crv[s] == r && stv[s] != kFrozen) {
                const bool inv = vmark[r] == stamp;
                S.state[r] = inv ? kInvalid : kValid;
                inv_mine |= inv;
            }
        }
        const bool any_inv = ballot(inv_mine) != 0ull;
        wave_sync();
        rounds++;
        if (MU && grow_all) {
            if (--mu_left == 0) break;
            continue;
        }
        if (!any_inv) {
            if (!MU || A.mu <= 0) break;
            grow_all = true;
            mu_left = A.mu;
        }
    }
    if (npc > KNP) { overflow(status); return; }

    // Largest cluster in columns (only when the caller asked for the info record): every
    // clustered fault counts once at the final root of its first detector's local row.  The
    // selection array is free after the last round (osd_e_clusters does not use it).
    // With A.cstats the same counts also give the shot's cluster statistics.
    auto max_cluster_cols = [&](int ncl) -> int {
        if (!A.info && !A.cstats) return 0;
        uint32_t *cnt = (uint32_t *)S.sel;
        for (int r = lane; r < K; r += 64) cnt[r] = 0u;
        wave_sync();
        for (int j = lane; j < n; j += 64)
            if (in_col(S.incol, j)) atomicAdd(&cnt[find_root(S.croot, S.loc[g.row_idx(g.col_ptr(j))])], 1u);
        wave_sync();
        uint32_t mx = 0u, tot = 0u, sq = 0u;
        for (int r = lane; r < K; r += 64) {
            const uint32_t v = cnt[r];
            mx = v > mx ? v : mx;
            tot += v;
            sq += v * v;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const uint32_t o = (uint32_t)__shfl_xor((int)mx, off, 64);
            mx = o > mx ? o : mx;
            tot += (uint32_t)__shfl_xor((int)tot, off, 64);
            sq += (uint32_t)__shfl_xor((int)sq, off, 64);
        }
        if (A.cstats && lane == 0) A.cstats[shot] = qlsd_cluster_stats{ncl, (int)mx, (int)tot, (int)sq};
        return (int)mx;
    };

    // solve: seed rows carry s = 1, claimed rows s = 0; frozen clusters contribute nothing
    uint64_t as[W];
#pragma unroll
    for (int s = 0; s < W; s++) {
        const int r = s * 64 + lane;
        const bool seed = r < nseed && S.state[S.croot[r]] != kFrozen;
        as[s] = ballot(seed) & B.piv[s];
    }
    int ncl = 0;
    uint64_t x0[W];  // LSD-0 solution: pivot rows whose column is set
#pragma unroll
    for (int s = 0; s < W; s++) {
        const int r = s * 64 + lane;
        const bool is_root = r < nrows && S.croot[r] == r;
        ncl += __popcll(ballot(is_root));
        x0[s] = ballot(((B.piv[s] >> lane) & 1ull) && parity_C<W>(B, s, as));
    }
    if (!MU || A.mu <= 0) {
#pragma unroll
        for (int s = 0; s < W; s++) {
            if ((x0[s] >> lane) & 1ull) {
                const int col = S.colAt[s * 64 + lane];
                atomicOr(&S.cbit[col >> 5], 1u << (col & 31));
            }
        }
        // faults of frozen clusters stay zero: their pivot rows never enter `as`
        write_row();
        finish(status, ncl, max_cluster_cols(ncl));
        return;
    }
    if constexpr (MU) osd_e_clusters<W, KNP>(A, S, g, B, x0, nrows, npc, llr, lane);
    write_row();
    finish(status, ncl, max_cluster_cols(ncl));
}

// Per-wavefront LDS block of decode_shot (lsd_layout order) at `base`.
__device__ inline LsdLds carve_lsd(unsigned char *base, int m, int n, int K, bool keys_in_lds, bool with_mu,
                                   int knp = 0) {
    size_t offs[kLsdLayoutEntries];
    lsd_layout(m, n, K, keys_in_lds, with_mu, offs, knp);
    LsdLds S;
    S.keys = (uint32_t *)(base + offs[0]);
    S.sel = (uint64_t *)(base + offs[1]);
    S.lkey = (uint64_t *)(base + offs[2]);
    S.lroot = (int32_t *)(base + offs[3]);
    S.colAt = (int32_t *)(base + offs[4]);
    S.croot = (int32_t *)(base + offs[5]);
    S.rowOf = (int32_t *)(base + offs[6]);
    S.loc = (int32_t *)(base + offs[7]);
    S.claimer = (int32_t *)(base + offs[8]);
    S.incol = (uint32_t *)(base + offs[9]);
    S.state = (uint8_t *)(base + offs[10]);
    S.ctl = (int32_t *)(base + offs[11]);
    S.colNP = (int32_t *)(base + offs[12]);
    S.wq = (int64_t *)(base + offs[13]);
    S.zk = (uint64_t *)(base + offs[14]);
    S.tsel = (int32_t *)(base + offs[15]);
    S.tw = (int64_t *)(base + offs[16]);
    S.cand = (uint64_t *)(base + offs[17]);
    S.cbit = (uint32_t *)(base + offs[18]);
    return S;
}

}  // namespace

}  // namespace qlsd
