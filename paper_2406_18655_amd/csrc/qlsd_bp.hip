// Min-sum belief propagation, parallel (flooding) schedule, for many shots at once.
//
// Message rules (Hillmann et al., Sec. 4.3: min-sum with scaling alpha, parallel schedule):
//   check -> fault : r_{i->j} = (-1)^{s_i} * alpha * prod_{j' != j} sgn(q_{j'->i}) * min_{j' != j} |q_{j'->i}|
//   fault -> check : q_{j->i} = lambda_j + sum_{i' != i} r_{i'->j},  L_j = lambda_j + sum_i r_{i->j}
//   hard decision  : e_j = [L_j < 0]; a shot has converged once H e = s (tested after every iteration).
// Magnitudes of q and L are clamped to 2^64 so that 100 iterations cannot overflow float32.
//
// Design (MI355X): a workgroup owns S shot "slots" whose messages live entirely in LDS, slot after
// slot at a stride the host picks with a model of the LDS banks (bp_msg_stride), so the lanes that
// work on a few consecutive checks or faults across the slots spread over the banks.  Each loop
// iteration runs one check phase and one fault phase over the
// active slots only.  A slot whose shot converged (or ran out of iterations) is retired and
// immediately refilled from a global queue, so early-exiting shots never leave lanes idle; the
// number of work items shrinks only once the queue is empty.  HBM traffic is only the syndrome
// in, the correction out, and the posterior LLRs of shots that go on to LSD.
#include <algorithm>
#include <functional>
#include <cstring>
#include <type_traits>

#include "qlsd_internal.h"
#include "qlsd_lsd_dev.h"

namespace qlsd {

namespace {

constexpr float kClamp = 18446744073709551616.0f;  // 2^64

__device__ __forceinline__ float clampf(float x) { return __builtin_amdgcn_fmed3f(x, -kClamp, kClamp); }

struct BpLds {
    int SE, SN, PW;  // message stride per slot (chosen on the host, bp_msg_stride), posterior
                     // stride (odd); 32-bit words per slot of the syndrome / parity bit vectors
    int C;           // shots per queue chunk
    float *msg, *Lv, *lam;
    uint32_t *synw, *parw;
    int *act, *newk, *newq, *rk, *rshot, *rit, *rconv, *ctl;
    uint16_t *rp, *ci, *cp, *ce, *ri;
    uint4 *nt;       // regular codes: per fault, its 3 edge ids and 3 check keys (16 bits each; a
                     // check's key is (byte offset of its parity word) << 5 | bit) and its prior,
                     // so one 16-byte read gives everything a fault item needs
    uint8_t *stg;    // 2 chunk buffers of C syndromes (raw bytes)
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }
__host__ __device__ inline int odd_stride(int x) { return x | 1; }
// Graph tables at the start of the BP block.  reg: the per-fault packed record (BpLds::nt) takes
// the place of the CSC edge-id table.
__host__ __device__ inline size_t tables_bytes(int m, int n, int E, bool reg) {
    return reg ? sizeof(uint4) * (size_t)n + align16(sizeof(uint16_t) * ((size_t)m + 1 + E + n + 1 + E))
               : align16(sizeof(uint16_t) * ((size_t)m + 1 + E + n + 1 + 2 * (size_t)E));
}

constexpr int kSlotArrays = 7;   // int arrays of S entries in the slot-state block
constexpr int kCtl = 16;         // control words

template <bool REG>
__device__ inline BpLds carve_bp(unsigned char *base, int m, int n, int E, int S, int SE) {
    BpLds L;
    L.SE = SE;
    L.SN = odd_stride(n);
    L.PW = (m + 31) / 32;
    L.C = S;
    // graph tables first: they stay valid for LSD once the slots are retired (fused kernel)
    size_t off = 0;
    L.nt = nullptr;
    L.ce = nullptr;
    if (REG) { L.nt = (uint4 *)base; off += sizeof(uint4) * n; }
    L.rp = (uint16_t *)(base + off); off += sizeof(uint16_t) * (m + 1);
    L.ci = (uint16_t *)(base + off); off += sizeof(uint16_t) * E;
    L.cp = (uint16_t *)(base + off); off += sizeof(uint16_t) * (n + 1);
    if (!REG) { L.ce = (uint16_t *)(base + off); off += sizeof(uint16_t) * E; }
    L.ri = (uint16_t *)(base + off);
    off = tables_bytes(m, n, E, REG);
    L.msg = (float *)(base + off); off += sizeof(float) * (size_t)L.SE * S;
    L.Lv = (float *)(base + off); off += sizeof(float) * (size_t)L.SN * S;
    L.lam = (float *)(base + off); off += sizeof(float) * n;
    L.synw = (uint32_t *)(base + off); off += sizeof(uint32_t) * (size_t)L.PW * S;
    L.parw = (uint32_t *)(base + off); off += sizeof(uint32_t) * (size_t)L.PW * S;
    int *ip = (int *)(base + off);
    L.act = ip; L.newk = ip + S; L.newq = ip + 2 * S;
    L.rk = ip + 3 * S; L.rshot = ip + 4 * S; L.rit = ip + 5 * S; L.rconv = ip + 6 * S;
    L.ctl = ip + kSlotArrays * S;
    off += sizeof(int) * ((size_t)kSlotArrays * S + kCtl);
    L.stg = (uint8_t *)(base + off);
    return L;
}

// The blocks of one active slot.  In each iteration a thread serves a single active slot per
// phase (fault phase: slot t mod A, rows t div A, + R, + 2R, ... with R = NT div A; check phase:
// the same over wavefronts 1.., with t - 64 and NT - 64), so the slot's block addresses are
// computed once per iteration rather than once per work item.
struct SlotView {
    float *msg;           // messages, one per edge (q after the fault phase, r after the check phase)
    float *Lv;            // posteriors
    uint32_t *parw;       // parity of the hard decision, one bit per check
    const uint32_t *synw; // syndrome bits
};

// Fault (variable-node) update of fault j in one active slot: posterior, exclusive sums, and
// the hard decision's contribution to every check's parity.  A fresh slot's messages were zeroed
// when its shot arrived, so in its first pass the incoming check messages are zero and the
// posterior is the prior, with no special case.  REG: every column has exactly CW = 3 edges, and
// one 16-byte read of the packed fault record gives the edge ids, check keys and prior.
template <int CW, bool REG>
struct FaultItem {
    static_assert(!REG || CW == 3, "the packed fault record describes 3 edges");
    float r[CW];
    int eid[CW];
    uint32_t chk[CW];  // REG: the fault's check keys (parity word byte offset << 5 | bit)
    int c0, cw, j;
    float lam;
    __device__ __forceinline__ void load(const BpLds &L, const SlotView &V, int j_) {
        j = j_;
        if constexpr (REG) {
            const uint4 rec = L.nt[j];
            eid[0] = (int)(rec.x & 0xffffu);
            eid[1] = (int)(rec.x >> 16);
            eid[2] = (int)(rec.y & 0xffffu);
            chk[0] = rec.y >> 16;
            chk[1] = rec.z & 0xffffu;
            chk[2] = rec.z >> 16;
            lam = __uint_as_float(rec.w);
            c0 = j * CW;
            cw = CW;
        } else {
            lam = L.lam[j];
            c0 = L.cp[j];
            cw = L.cp[j + 1] - c0;
#pragma unroll
            for (int u = 0; u < CW; u++) eid[u] = u < cw ? (int)L.ce[c0 + u] : 0;
        }
#pragma unroll
        for (int u = 0; u < CW; u++) {
            const float v = V.msg[eid[u]];  // padding entries read edge 0 of the slot
            r[u] = (REG || u < cw) ? v : 0.f;
        }
    }
    __device__ __forceinline__ void store(const BpLds &L, const SlotView &V, bool count_parity) const {
        float pre[CW + 1];
        pre[0] = lam;
#pragma unroll
        for (int u = 0; u < CW; u++) pre[u + 1] = pre[u] + r[u];
        if constexpr (REG) {
            // The suffix sum starts at the last edge rather than at +0: the same values, since a
            // prefix sum is -0 only if the prior is, and log((1-p)/p) never rounds to -0.
            float suf = r[CW - 1];
            V.msg[eid[CW - 1]] = clampf(pre[CW - 1]);
#pragma unroll
            for (int u = CW - 2; u >= 0; u--) {
                V.msg[eid[u]] = clampf(pre[u] + suf);
                suf += r[u];
            }
        } else {
            float suf = 0.f;
#pragma unroll
            for (int u = CW - 1; u >= 0; u--) {
                if (u < cw) {
                    V.msg[eid[u]] = clampf(pre[u] + suf);
                    suf += r[u];
                }
            }
        }
        const float Lt = clampf(pre[CW]);  // padding entries add exact zeros
        V.Lv[j] = Lt;
        if (count_parity && Lt < 0.f) {
#pragma unroll
            for (int u = 0; u < CW; u++) {
                if (REG) {
                    atomicXor((uint32_t *)((unsigned char *)V.parw + (chk[u] >> 5)), 1u << (chk[u] & 31));
                } else if (u < cw) {
                    const int i = L.ri[c0 + u];
                    atomicXor(V.parw + (i >> 5), 1u << (i & 31));
                }
            }
        }
    }
};

// Check update of check i in one active slot (min-sum with the syndrome sign).  REG: every
// row has exactly RW edges.
template <int RW, bool REG>
struct CheckItem {
    float q[RW];
    int e0, rw;
    uint32_t sb;
    __device__ __forceinline__ void load(const BpLds &L, const SlotView &V, int i) {
        e0 = REG ? __umul24(i, RW) : L.rp[i];
        rw = REG ? RW : L.rp[i + 1] - e0;
        sb = (V.synw[i >> 5] >> (i & 31)) & 1u;
#pragma unroll
        for (int u = 0; u < RW; u++) q[u] = (REG || u < rw) ? V.msg[e0 + u] : INFINITY;
    }
    // pinf / ninf: +inf and -inf held opaque to the compiler (see the kernel)
    __device__ __forceinline__ void store(const BpLds &L, const SlotView &V, float alpha, float pinf,
                                          float ninf) const {
        uint32_t sg = sb << 31;
        float mn1 = pinf, mn2 = pinf;
        // min(x, y) as med3(x, y, -inf): the same value for these non-NaN magnitudes, in one
        // instruction (fminf costs a canonicalising one per operand)
#pragma unroll
        for (int u = 0; u < RW; u++) {
            sg ^= __float_as_uint(q[u]);
            const float a = fabsf(q[u]);
            mn2 = __builtin_amdgcn_fmed3f(mn1, mn2, a);
            mn1 = __builtin_amdgcn_fmed3f(mn1, a, ninf);
        }
        float m1 = alpha * mn1, m2 = alpha * mn2;
        // keep the two products (otherwise the multiply is repeated after every select)
        asm volatile("" : "+v"(m1), "+v"(m2));
#pragma unroll
        for (int u = 0; u < RW; u++) {
            if (REG || u < rw) {
                const float mag = (fabsf(q[u]) == mn1) ? m2 : m1;
                const uint32_t sgn = (sg ^ __float_as_uint(q[u])) & 0x80000000u;
                V.msg[e0 + u] = __uint_as_float(__float_as_uint(mag) | sgn);
            }
        }
    }
};

// Control words (L.ctl), written by slot management for every wavefront: [0] retired, [1] fresh,
// [2] active this iteration; [3] retired without converging; [5] request pending; [6] load scheduled (base, -1 none), [7] its
// count, [8] its buffer.  Before the loop: [9] queue exhausted, [10] / [11] base (-1: none) and
// count of the first chunk.
// Hand-over between workgroups in the fused kernel.  The L2 caches of different XCDs are not
// coherent with each other, so every word that crosses workgroups during the kernel -- the LLR
// row of an unsolved shot, its list entry, the counters -- is written and read only with
// device-scope read-modify-write atomics, which are performed at the device's point of
// coherence: a poll never sees a line cached by its own XCD, and no write leaves a dirty line
// whose later write-back could restore stale neighbouring words.  A publisher's row atomics
// complete before the barrier that precedes the list entries naming them; a consumer's row
// reads are issued after, and depend on, the entry it read.  The correction row and info record
// of an unsolved shot are written only by the LSD side.
// A compare-and-swap whose new value equals its compare value never changes memory and always
// returns the word from the point of coherence (an idempotent add would be turned into a load).
__device__ __forceinline__ int poll_agent(int *p) { return atomicCAS(p, 0, 0); }

// How long a fused LSD wavefront waits without work before it leaves (wall-clock ticks of 10 ns).
// Leaving only moves work to the stand-alone LSD launch after the kernel, so the wait is short:
// long enough to pick up shots other workgroups publish in a steady stream, short enough that
// waiting wavefronts do not keep polling while the last BP workgroups run (at low noise there
// are only a few hundred LSD shots per batch).
constexpr unsigned long long kFuseLingerTicks = 2000;  // 20 us
// A wavefront that holds a ticket waits for its entry until the entry can no longer come (every
// BP workgroup done with fewer entries) or nothing happened for this long -- a bound that only
// matters if the grid is not co-resident (e.g. concurrent serving lanes).  Such tickets are few:
// they come from races between wavefronts that saw the same published entry.
constexpr unsigned long long kFuseTicketTicks = 20000;  // 200 us

// Everything a fused LSD wavefront does between two shots, as one call that the whole wavefront
// makes with uniform control flow: mark entry done_h decoded (done_h >= 0), then take a ticket h
// for a published entry and wait for it.  A ticket is taken only while published entries exceed
// the tickets handed out (a race can still hand out one beyond them; that ticket waits too).
// Returns {shot, h}, uniform across the wavefront, or shot = -1 once no work is left (every BP
// workgroup done and the list exhausted), or none came for kFuseLingerTicks (no ticket held) or
// kFuseTicketTicks (ticket held).  The lane-0 atomics
// live here, not in the caller's loop, because the compiler does not guarantee that a wavefront
// reconverges after a lane-0 region inside a loop: it may split lane 0 off at the loop latch and
// run the loop body (a whole LSD shot, which needs all 64 lanes) with the other lanes only.  A
// call returns with the caller's execution mask.
__device__ __noinline__ int2 fuse_step(int *list, int *next_item, int *bp_done, int *tail, int *lsd_done, int nwg,
                                       int B, int done_h, int done_shot) {
    const int lane = threadIdx.x & 63;
    if (lane == 0 && done_h >= 0) {
        atomicExch(list + done_h, ~done_shot);  // the stand-alone launch skips it
        atomicAdd(lsd_done, 1);
    }
    unsigned long long t0 = wall_clock64();
    int nap = 1;
    int h = -1;  // ticket held (wave-uniform)
    for (int poll = 0;; poll++) {
        int v = -1, tl = 0, nx = 0, done = 0;
        if (lane == 0) {
            if (h >= 0) {
                v = poll_agent(list + h);
                if (v < 0 && (poll & 3) == 3) {
                    done = poll_agent(bp_done);
                    tl = poll_agent(tail);
                }
            } else {
                tl = poll_agent(tail);
                nx = poll_agent(next_item);
                if (tl > nx) v = -2 - atomicAdd(next_item, 1);  // a ticket: -2 - h
                else done = poll_agent(bp_done);
            }
        }
        v = __builtin_amdgcn_readfirstlane(v);
        if (h >= 0) {
            if (v >= 0) return make_int2(v, h);
            // entry h can no longer come: every BP workgroup done, fewer entries
            if (__builtin_amdgcn_readfirstlane(done) >= nwg && __builtin_amdgcn_readfirstlane(tl) <= h)
                return make_int2(-1, h);
        } else if (v <= -2) {
            h = -2 - v;
            if (h >= B) return make_int2(-1, h);  // at most B entries
            t0 = wall_clock64();
            nap = 1;
            poll = -1;
            continue;  // poll the entry at once: it is published or about to be
        } else if (__builtin_amdgcn_readfirstlane(done) >= nwg) {
            // every BP workgroup is done: the list is final
            int tl2 = 0, nx2 = 0;
            if (lane == 0) {
                tl2 = poll_agent(tail);
                nx2 = poll_agent(next_item);
            }
            if (__builtin_amdgcn_readfirstlane(tl2) <= __builtin_amdgcn_readfirstlane(nx2)) return make_int2(-1, -1);
            continue;
        }
        if (wall_clock64() - t0 > (h >= 0 ? kFuseTicketTicks : kFuseLingerTicks)) return make_int2(-1, h);
        for (int k = 0; k < nap; k++) __builtin_amdgcn_s_sleep(64);  // 4096 cycles, ~1.7 us each
        nap = min(nap * 2, 4);
    }
}

// LSDW = 0: BP only.  LSDW = W > 0: BP, then LSD (decode_shot<W>) on published shots; OVF: the
// code has more checks than the 64 W local rows, and a shot whose clusters outgrow them is listed
// for the overflow kernels (compiled in only where it can happen: it costs registers).  At most 128
// VGPRs (4 wavefronts per SIMD), so that four BP workgroups fit on a CU.
template <int MAXRW, int MAXCW, bool REG, int LSDW, bool OVF = false>
__global__ __launch_bounds__(kBpThreads) __attribute__((amdgpu_waves_per_eu(4)))
void bp_lds_kernel(BpArgs args, FuseArgs f) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = threadIdx.x, NT = blockDim.x;
    const int lane = t & 63, wave = t >> 6;
    const int m = args.g.m, n = args.g.n, E = args.g.nnz, S = args.S;
    BpLds L = carve_bp<REG>(smem, m, n, E, S, args.SE);
    const int C = L.C;

    for (int x = t; x <= m; x += NT) L.rp[x] = (uint16_t)args.g.row_ptr[x];
    for (int x = t; x < E; x += NT) L.ci[x] = (uint16_t)args.g.col_idx[x];
    for (int x = t; x <= n; x += NT) L.cp[x] = (uint16_t)args.g.col_ptr[x];
    if constexpr (REG) {
        for (int x = t; x < n; x += NT) {
            uint32_t e[3], c[3];
            for (int u = 0; u < 3; u++) {
                const uint32_t i = (uint32_t)args.g.row_idx[x * 3 + u];
                e[u] = (uint32_t)args.g.col_edge[x * 3 + u];
                c[u] = (i >> 5) << 7 | (i & 31);  // fits 16 bits: m <= 16384 on this path
            }
            L.nt[x] = make_uint4(e[0] | e[1] << 16, e[2] | c[0] << 16, c[1] | c[2] << 16, __float_as_uint(args.lam[x]));
        }
    } else {
        for (int x = t; x < E; x += NT) L.ce[x] = (uint16_t)args.g.col_edge[x];
    }
    for (int x = t; x < E; x += NT) L.ri[x] = (uint16_t)args.g.row_idx[x];
    for (int x = t; x < n; x += NT) L.lam[x] = args.lam[x];
    for (int x = t; x < S * L.PW; x += NT) { L.parw[x] = 0u; L.synw[x] = 0u; }
    // first chunk: fetched synchronously into staging buffer 0
    if (t == 0) {
        const int b0 = atomicAdd(args.next_shot, C);
        const int c0 = max(0, min(C, args.B - b0));
        L.ctl[9] = b0 + C >= args.B;
        L.ctl[10] = c0 > 0 ? b0 : -1;
        L.ctl[11] = c0;
    }
    __syncthreads();
    if (L.ctl[10] >= 0) {
        const int b0 = L.ctl[10], c0 = L.ctl[11];
        for (int x = t; x < c0 * m; x += NT) L.stg[x] = args.syn[(size_t)b0 * m + x];
    }
    __syncthreads();

    const float alpha = args.alpha;
    // infinities the compiler cannot see through, so the check update's med3 minima stay med3
    // (with a known -inf it turns them back into fminf, which canonicalises its operands)
    float pinf = INFINITY, ninf = -INFINITY;
    asm volatile("" : "+v"(pinf), "+v"(ninf));
    const int T = args.max_iter;
    const int PW = L.PW;
    const uint64_t lt = (1ull << lane) - 1ull;
    // fused: BP wavefronts issue ahead of the LSD wavefronts of drained workgroups on the same CU
    // (the last BP shots gate the last LSD shots)
    if constexpr (LSDW > 0) __builtin_amdgcn_s_setprio(2);
    // Queue state, held in wavefront 0's registers (uniform across its lanes; no other wavefront
    // reads it): staging buffer k holds shots [qb_k, qb_k + qc_k) (qb_k = -1: free, -2: drained
    // this iteration, still readable); cur / cursor: next staged shot; pending: a chunk request
    // issued one iteration ago (its base in req); exhausted: no shots left to request.  A slot's
    // shot and iteration count live in the lane of wavefront 0 that manages the slot.
    int qb0 = L.ctl[10], qc0 = L.ctl[11], qb1 = -1, qc1 = 0;
    int q_cur = 0, q_cursor = 0, q_pending = 0, q_exh = L.ctl[9];
    int req_v = 0;   // lane 0: base returned by the request in flight (read once it has landed)
    int q_sz = C;    // shots asked for by that request
    int q_seen = qb0 >= 0 ? qb0 : args.B;  // base of the latest chunk landed here (queue position)
    int my_shot = -1, my_it = 0;
    // the check phase's rows and slot (wavefronts 1..), kept from one loop pass to the next
    int rc0 = 1 << 30, Rc = NT;
    SlotView Vc;
    Vc.msg = L.msg;
    Vc.synw = L.synw;

    for (;;) {
        // ---- slot management (wavefront 0, one lane per slot): test convergence (parity of the
        // last hard decision against the syndrome), retire converged or exhausted shots, give
        // free slots the next staged shots, list the active slots, keep the queue pipeline full.
        // Meanwhile wavefronts 1.. run the check phase of the iteration whose fault phase just
        // ended: slot management needs only that fault phase's parity words, and the check phase
        // reads no word that slot management writes (its slot's blocks are in registers).
        if (wave == 0) {
            const bool valid = lane < S;
            int shot = valid ? my_shot : -1;
            int it = valid ? my_it : 0;
            const bool active = shot >= 0;
            bool sat = active;
            if (active) {
                for (int w = 0; w < PW; w++) {
                    sat &= L.parw[lane * PW + w] == L.synw[lane * PW + w];
                    L.parw[lane * PW + w] = 0u;
                }
            }
            const bool conv = active && it >= 1 && sat;
            const bool retire = active && ((args.early_exit && conv) || it >= T);
            const bool need = valid && (!active || retire);
            const uint64_t rmask = __ballot(retire);
            const uint64_t fmask_unsolved = __ballot(retire && !conv);
            if (retire) {
                const int p = __popcll(rmask & lt);
                L.rk[p] = lane;
                L.rshot[p] = shot;
                L.rit[p] = it;
                L.rconv[p] = conv ? 1 : 0;
            }
            // staged shots: the rest of the current buffer, then the other buffer if loaded
            const int cur = q_cur, cursor = q_cursor;
            const int cbase = cur ? qb1 : qb0, ccount = cur ? qc1 : qc0;
            const int obase = cur ? qb0 : qb1, ocount = cur ? qc0 : qc1;
            const int avail0 = cbase >= 0 ? ccount - cursor : 0;
            const int avail1 = obase >= 0 ? ocount : 0;
            const uint64_t nmask = __ballot(need);
            const int r = __popcll(nmask & lt);
            bool fresh = false;
            if (need) {
                if (r < avail0) {
                    shot = cbase + cursor + r;
                    fresh = true;
                    L.newq[r] = cur * C + cursor + r;
                } else if (r - avail0 < avail1) {
                    shot = obase + (r - avail0);
                    fresh = true;
                    L.newq[r] = (1 - cur) * C + (r - avail0);
                } else {
                    shot = -1;
                }
                it = 0;
            } else if (active) {
                it = it + 1;
            }
            if (valid) { my_shot = shot; my_it = it; }
            const uint64_t fmask = __ballot(fresh);
            const int nfresh = __popcll(fmask);
            if (fresh) L.newk[r] = lane;  // fresh lanes are exactly the first nfresh needing ones
            const bool on = valid && shot >= 0;
            const uint64_t amask = __ballot(on);
            if (on) {
                const int a = __popcll(amask & lt);
                L.act[a] = lane;
            }
            // buffers drained last iteration are free now
            if (qb0 == -2) qb0 = -1;
            if (qb1 == -2) qb1 = -1;
            auto set_buf = [&](int k, int base, int cnt) {
                if (k) { qb1 = base; qc1 = cnt; } else { qb0 = base; qc0 = cnt; }
            };
            // advance the cursor; a buffer drained now stays readable for this iteration
            int ncur = cur, ncursor = cursor;
            if (nfresh < avail0) {
                ncursor = cursor + nfresh;
            } else if (cbase >= 0) {
                set_buf(cur, -2, 0);
                if (obase >= 0) {
                    ncur = 1 - cur;
                    ncursor = nfresh - avail0;
                    if (ncursor >= ocount) {
                        set_buf(ncur, -2, 0);
                        ncursor = 0;
                    }
                } else {
                    ncursor = 0;
                }
            } else if (obase >= 0) {
                // the current buffer holds nothing (drained or free): every fresh shot came
                // from the other buffer, which becomes the current one
                ncur = 1 - cur;
                ncursor = nfresh;
                if (ncursor >= ocount) {
                    set_buf(ncur, -2, 0);
                    ncursor = 0;
                }
            }
            q_cur = ncur;
            q_cursor = ncursor;
            // a request issued one iteration ago has landed: stage that chunk now
            int ldb = -1, ldc = 0, ldbuf = 0;
            if (q_pending) {
                q_pending = 0;
                const int req = __builtin_amdgcn_readfirstlane(req_v);
                const int cnt = max(0, min(q_sz, args.B - req));
                if (req + q_sz >= args.B) q_exh = 1;
                q_seen = req;
                if (cnt > 0) {
                    // a free buffer exists: requests are only issued when one is free
                    const int dst = (ncur ? qb1 : qb0) == -1 ? ncur : 1 - ncur;
                    set_buf(dst, req, cnt);
                    if (dst == ncur) q_cursor = 0;
                    ldb = req;
                    ldc = cnt;
                    ldbuf = dst;
                }
            }
            // keep one request in flight while a buffer is free and shots remain; requests shrink
            // as the queue drains (about a quarter of each workgroup's share of what is left, at
            // most a chunk), so no workgroup still holds full chunks when the others run dry
            // One kernel with LSD: odd-numbered workgroups stop taking new shots once less than a
            // fifth of the batch is left and turn to LSD while the others finish BP, so LSD starts
            // before the whole grid drains (the shared queue hands their share to the others).
            const bool lsd_early = LSDW > 0 && (blockIdx.x & 1) == 1 && (long long)(args.B - q_seen) * 5 < (long long)args.B;
            if (!q_exh && (qb0 == -1 || qb1 == -1) && !lsd_early) {
                q_sz = max(1, min(C, (args.B - q_seen) / (4 * (int)gridDim.x)));
                if (lane == 0) req_v = atomicAdd(args.next_shot, q_sz);
                q_pending = 1;
            }
            if (lane == 0) {
                L.ctl[0] = (int)__popcll(rmask);
                L.ctl[3] = (int)__popcll(fmask_unsolved);
                L.ctl[1] = nfresh;
                L.ctl[2] = (int)__popcll(amask);
                L.ctl[5] = q_pending;
                L.ctl[6] = ldb;
                L.ctl[7] = ldc;
                L.ctl[8] = ldbuf;
            }
        } else {
            // ---- check phase: min-sum messages, one item per thread at a time
            for (int i = rc0; i < m; i += Rc) {
                CheckItem<MAXRW, REG> it;
                it.load(L, Vc, i);
                it.store(L, Vc, alpha, pinf, ninf);
            }
        }
        __syncthreads();
        const int nret = L.ctl[0], nfresh = L.ctl[1], A = L.ctl[2], nunsolved = L.ctl[3];
        const int ldb = L.ctl[6], ldc = L.ctl[7], ldbuf = L.ctl[8];
        const bool pending = L.ctl[5] != 0;
        // this thread's active slot for the fault phase of the iteration: t = r0 * A + a with
        // r0 < Rs = NT div A (the division by reciprocal is exact for t < 256, A <= 128); the
        // NT mod A threads past Rs * A serve no slot
        int r0 = 1 << 30, Rs = NT;
        SlotView V;
        {
            int a = 0;
            if (A > 0) {
                const float rA = __builtin_amdgcn_rcpf((float)A);
                Rs = (int)(((float)NT + 0.5f) * rA);
                const int q = (int)(((float)t + 0.5f) * rA);
                if (q < Rs) {
                    r0 = q;
                    a = t - q * A;
                }
            }
            const int k = L.act[a];
            V.msg = L.msg + k * L.SE;
            V.Lv = L.Lv + k * L.SN;
            V.parw = L.parw + k * PW;
            V.synw = L.synw + k * PW;
        }
        // the same for the check phase, over wavefronts 1.. (tc = t - 64 = rc0 * A + a)
        {
            int a = 0;
            rc0 = 1 << 30;
            Rc = NT - 64;
            if (A > 0 && wave > 0) {
                const float rA = __builtin_amdgcn_rcpf((float)A);
                Rc = (int)(((float)(NT - 64) + 0.5f) * rA);
                const int q = (int)(((float)(t - 64) + 0.5f) * rA);
                if (q < Rc) {
                    rc0 = q;
                    a = (t - 64) - q * A;
                }
            }
            const int k = L.act[a];
            Vc.msg = L.msg + k * L.SE;
            Vc.synw = L.synw + k * PW;
        }

        // ---- outputs of retired shots (coalesced rows), staging of the next chunk, and the
        // syndromes of fresh shots (from staging, packed into bit words by wavefront ballots)
        // The chunk that landed goes to a buffer no shot reads before the next slot management:
        // its loads are issued here and their LDS stores wait until after the fault phase, so the
        // HBM round trip overlaps that phase instead of stalling every thread at the next barrier
        // (dwords held in registers when rows are 4-byte aligned and the chunk fits; else a copy).
        constexpr int kPre = 4;
        uint32_t pre[kPre];
        const int nw = ldc * m / 4;
        const bool pre_ok = ldb >= 0 && (m & 3) == 0 && (((uintptr_t)args.syn) & 3) == 0 && nw <= kPre * NT;
        if (pre_ok) {
            const uint32_t *src = (const uint32_t *)(args.syn + (size_t)ldb * m);
#pragma unroll
            for (int q = 0; q < kPre; q++) {
                const int x = t + q * NT;
                pre[q] = x < nw ? src[x] : 0u;
            }
        } else if (ldb >= 0) {
            uint8_t *dst = L.stg + (size_t)ldbuf * C * m;
            const uint8_t *src = args.syn + (size_t)ldb * m;
            for (int x = t; x < ldc * m; x += NT) dst[x] = src[x];
        }
        // Outputs are written by wavefronts 1.. only: wavefront 0 then has no global stores in
        // flight when slot management waits for its queue request (one counter covers both).
        for (int r = 0; r < nret && wave > 0; r++) {
            const int k = L.rk[r], shot = L.rshot[r];
            const bool conv = L.rconv[r] != 0;
            const size_t row = (size_t)shot * n;
            const bool write_corr = args.corr && (LSDW == 0 || conv);  // fused: LSD writes the rest
            for (int j = t - 64; j < n; j += NT - 64) {
                const float Lj = L.Lv[k * L.SN + j];
                if (write_corr) args.corr[row + j] = Lj < 0.f ? 1 : 0;
                if (args.llr_out) args.llr_out[row + j] = Lj;
                if (!conv && args.llr_lsd) {
                    if (LSDW > 0) atomicExch((int *)args.llr_lsd + row + j, __float_as_int(Lj));
                    else args.llr_lsd[row + j] = Lj;
                }
            }
            if (t == 64) {
                if (args.info && (LSDW == 0 || conv)) {
                    qlsd_shot_info inf;
                    inf.status = conv ? QLSD_ST_BP_CONVERGED : 0;
                    inf.reserved = 0;
                    inf.bp_iters = (int16_t)L.rit[r];
                    inf.n_clusters = 0;
                    inf.rounds = 0;
                    inf.max_cluster_cols = 0;
                    args.info[shot] = inf;
                }
                if (args.lsd_flag) args.lsd_flag[shot] = conv ? 0 : 1;
            }
        }
        if constexpr (LSDW > 0) {
            // publish the unsolved shots: their LLR rows and info records reach device scope
            // before the list entries that name them
            if (nunsolved > 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (wave > 0) __builtin_amdgcn_s_waitcnt(0);  // this thread's row atomics have completed
                __syncthreads();
                if (t == 64) {
                    int pos = atomicAdd(f.tail, nunsolved);
                    for (int r = 0; r < nret; r++)
                        if (!L.rconv[r]) atomicExch(f.list_w + pos++, L.rshot[r]);
                }
            }
        }
        for (int fi = wave; fi < nfresh; fi += NT / 64) {
            const int k = L.newk[fi];
            const uint8_t *sq = L.stg + (size_t)L.newq[fi] * m;
            float *mz = L.msg + k * L.SE;  // no incoming check messages yet
            for (int e = lane; e < E; e += 64) mz[e] = 0.f;
            for (int i0 = 0; i0 < m; i0 += 64) {
                const int i = i0 + lane;
                const uint64_t bits = __ballot(i < m && (sq[i] & 1));
                if (lane == 0) {
                    L.synw[k * PW + (i0 >> 5)] = (uint32_t)bits;
                    if ((i0 >> 5) + 1 < PW) L.synw[k * PW + (i0 >> 5) + 1] = (uint32_t)(bits >> 32);
                }
            }
        }
        if (A == 0 && !pending && ldb < 0) break;
        __syncthreads();

        // ---- fault phase (fresh slots start from q = lambda, i.e. zero incoming messages); one
        // item per thread at a time (more items in flight per thread measured slower)
        for (int j = r0; j < n; j += Rs) {
            FaultItem<MAXCW, REG> it;
            it.load(L, V, j);
            it.store(L, V, true);
        }
        if (pre_ok) {
            uint32_t *dst = (uint32_t *)(L.stg + (size_t)ldbuf * C * m);
#pragma unroll
            for (int q = 0; q < kPre; q++) {
                const int x = t + q * NT;
                if (x < nw) dst[x] = pre[q];
            }
        }
        __syncthreads();
        // (the check phase of this iteration runs at the top of the next pass)
    }

    if constexpr (LSDW > 0) {
        // ---- LSD on published shots: the slot arrays are dead, the graph tables stay
        __syncthreads();
        if (t == 0) atomicAdd(f.bp_done, 1);  // after this workgroup's last reservation
        if (wave >= f.lsd_waves) return;
        __builtin_amdgcn_s_setprio(0);
        constexpr int K = 64 * LSDW;
        unsigned char *lbase = smem + tables_bytes(m, n, E, REG) + (size_t)wave * f.lsd.wave_bytes;
        const LsdLds S2 = carve_lsd(lbase, m, n, K, f.lsd.keys_in_lds != 0, false);  // LSD-0 only
        GView<true> gv;
        gv.rp = L.rp; gv.ci = L.ci; gv.cp = L.cp; gv.ri = L.ri;
        gv.max_cw = args.g.max_cw;
        const int nwg = (int)gridDim.x;
        // no lane-dependent branch in this loop: see fuse_step
        int done_h = -1, done_shot = 0;
        for (;;) {
            const int2 r = fuse_step(f.list_w, f.lsd.next_item, f.bp_done, f.tail, f.lsd_done, nwg, args.B, done_h,
                                     done_shot);
            const int shot = __builtin_amdgcn_readfirstlane(r.x);
            const int h = __builtin_amdgcn_readfirstlane(r.y);
            if (shot < 0) break;  // no entry h, or it is left to the stand-alone launch (the call
                                  // that returned it has marked the previous shot done)
            decode_shot<LSDW, false, decltype(gv), false, OVF>(f.lsd, S2, gv, shot, lane);  // LSD-0 only
            wave_sync();
            done_h = h;
            done_shot = shot;
        }
    }
}

// ------------------------------------------------------------------------------------------
// Large graphs (e.g. a 936 x 8800 detector error model): one workgroup per shot.  The shot's
// messages (one float per edge) and posteriors live in LDS; H is read from global memory
// (it is shared by every workgroup and stays in L2).  Threads run over faults in the fault
// phase and over checks in the check phase; the syndrome test is the same XOR-parity scheme.
// ------------------------------------------------------------------------------------------
template <int MAXRW, int MAXCW>
__global__ __launch_bounds__(kBpGraphThreads) void bp_graph_kernel(BpArgs args) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = threadIdx.x, NT = blockDim.x;
    const int m = args.g.m, n = args.g.n, E = args.g.nnz;
    const int PW = (m + 31) / 32;
    float *msg = (float *)smem;
    float *Lv = msg + E;
    uint32_t *synw = (uint32_t *)(Lv + n);
    uint32_t *parw = synw + PW;
    int *ctl = (int *)(parw + PW);
    const int32_t *row_ptr = args.g.row_ptr, *col_ptr = args.g.col_ptr;
    const int32_t *col_edge = args.g.col_edge, *row_idx = args.g.row_idx;
    const float alpha = args.alpha;
    const int T = args.max_iter;
    const int lane = t & 63, wave = t >> 6;

    for (;;) {
        if (t == 0) ctl[0] = atomicAdd(args.next_shot, 1);
        __syncthreads();
        const int shot = ctl[0];
        if (shot >= args.B) break;
        const uint8_t *syn = args.syn + (size_t)shot * m;
        for (int i0 = wave * 64; i0 < m; i0 += NT) {
            const int i = i0 + lane;
            const uint64_t bits = __ballot(i < m && (syn[i] & 1));
            if (lane == 0) {
                synw[i0 >> 5] = (uint32_t)bits;
                if ((i0 >> 5) + 1 < PW) synw[(i0 >> 5) + 1] = (uint32_t)(bits >> 32);
            }
        }
        for (int w = t; w < PW; w += NT) parw[w] = 0u;
        for (int e = t; e < E; e += NT) msg[e] = 0.f;  // r = 0: the first fault phase sets q = lambda
        __syncthreads();
        int it = 0;
        bool conv = false;
        for (;;) {
            // fault phase
            for (int j = t; j < n; j += NT) {
                const int c0 = col_ptr[j], cw = col_ptr[j + 1] - c0;
                float r[MAXCW];
                int eid[MAXCW];
#pragma unroll
                for (int u = 0; u < MAXCW; u++) {
                    eid[u] = u < cw ? col_edge[c0 + u] : 0;
                    r[u] = u < cw ? msg[eid[u]] : 0.f;
                }
                const float lam = args.lam[j];
                float pre[MAXCW + 1];
                pre[0] = lam;
#pragma unroll
                for (int u = 0; u < MAXCW; u++) pre[u + 1] = pre[u] + r[u];
                float suf = 0.f;
#pragma unroll
                for (int u = MAXCW - 1; u >= 0; u--) {
                    if (u < cw) {
                        msg[eid[u]] = clampf(pre[u] + suf);
                        suf += r[u];
                    }
                }
                const float Lt = clampf(pre[MAXCW]);
                Lv[j] = Lt;
                if (Lt < 0.f) {
                    for (int u = 0; u < cw; u++) {
                        const int i = row_idx[c0 + u];
                        atomicXor(parw + (i >> 5), 1u << (i & 31));
                    }
                }
            }
            __syncthreads();
            // syndrome test of the hard decision after iteration it (it >= 1)
            if (wave == 0) {
                bool ok = true;
                for (int w = lane; w < PW; w += 64) {
                    ok &= parw[w] == synw[w];
                    parw[w] = 0u;
                }
                const bool all = __ballot(!ok) == 0;
                if (lane == 0) ctl[1] = all ? 1 : 0;
            }
            __syncthreads();
            const bool sat = ctl[1] != 0;
            conv = it >= 1 && sat;
            if ((args.early_exit && conv) || it >= T) break;
            it++;
            // check phase
            for (int i = t; i < m; i += NT) {
                const int e0 = row_ptr[i], rw = row_ptr[i + 1] - e0;
                const uint32_t sb = (synw[i >> 5] >> (i & 31)) & 1u;
                float q[MAXRW];
#pragma unroll
                for (int u = 0; u < MAXRW; u++) q[u] = u < rw ? msg[e0 + u] : INFINITY;
                uint32_t sg = sb << 31;
                float mn1 = INFINITY, mn2 = INFINITY;
#pragma unroll
                for (int u = 0; u < MAXRW; u++) {
                    sg ^= __float_as_uint(q[u]);
                    const float a = fabsf(q[u]);
                    mn2 = __builtin_amdgcn_fmed3f(mn1, mn2, a);
                    mn1 = fminf(mn1, a);
                }
                const float m1 = alpha * mn1, m2 = alpha * mn2;
#pragma unroll
                for (int u = 0; u < MAXRW; u++) {
                    if (u < rw) {
                        const float mag = (fabsf(q[u]) == mn1) ? m2 : m1;
                        const uint32_t sgn = (sg ^ __float_as_uint(q[u])) & 0x80000000u;
                        msg[e0 + u] = __uint_as_float(__float_as_uint(mag) | sgn);
                    }
                }
            }
            __syncthreads();
        }
        // outputs
        const size_t row = (size_t)shot * n;
        for (int j = t; j < n; j += NT) {
            const float Lj = Lv[j];
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
            if (args.lsd_flag) args.lsd_flag[shot] = conv ? 0 : 1;
        }
        __syncthreads();
    }
}

}  // namespace

// Codes decoded by the fully unrolled instantiation (every row weight 6, every column weight 3;
// at most 16384 checks, so a check key of the packed fault record fits 16 bits).
static bool bp_regular63(const DevGraph &g) {
    return g.min_rw == g.max_rw && g.min_cw == g.max_cw && g.max_rw == 6 && g.max_cw == 3 && g.m <= 16384;
}

size_t bp_tables_bytes(const DevGraph &g) { return tables_bytes(g.m, g.n, g.nnz, bp_regular63(g)); }

size_t bp_lds_bytes(const DevGraph &g, int S, int SE) {
    // carve_bp's order: graph tables, messages, posteriors, priors, bit vectors, slot state, staging
    const size_t PW = ((size_t)g.m + 31) / 32;
    size_t b = bp_tables_bytes(g);
    b += sizeof(float) * ((size_t)SE * S + (size_t)odd_stride(g.n) * S + g.n);
    b += sizeof(uint32_t) * 2 * PW * S;
    b += sizeof(int) * ((size_t)kSlotArrays * S + kCtl);
    b += (size_t)2 * S * g.m;  // two staging buffers of S syndromes
    return align16(b);
}

int bp_min_stride(const DevGraph &g) { return odd_stride(g.nnz); }

// LDS cycles of one pass of the slot kernel over every check and every fault with all S slots
// active, in a model of the LDS as 32 banks of 4 bytes serving a wavefront in two halves of 32
// lanes: a message access costs, per half, the largest number of its lanes whose words fall in one
// bank.  Lane t of a phase serves slot t mod S of check (or fault) t div S, so the lanes of a
// wavefront read edge u of a few consecutive checks (faults) in every slot, at slot * SE + edge.
static long long bp_bank_cycles(const int32_t *row_ptr, const int32_t *col_ptr, const int32_t *col_edge, int m,
                                int n, int max_rw, int max_cw, int S, int SE) {
    long long cyc = 0;
    int bank[32];
    auto pass = [&](int items, int first_thread, int max_w, auto addr) {
        const int NT = kBpThreads - first_thread;  // threads of the phase
        const int R = NT / S;                      // items per step
        for (int it = 0; it < items; it += R)
            for (int w0 = 0; w0 < NT; w0 += 64)
                for (int u = 0; u < max_w; u++)
                    for (int h = 0; h < 64; h += 32) {
                        std::fill(bank, bank + 32, 0);
                        int mx = 0;
                        for (int l = h; l < h + 32; l++) {
                            const int t = w0 + l, r = t / S, a = t % S, x = it + r;
                            if (r >= R || x >= items) continue;
                            const long long ad = addr(x, u);
                            if (ad < 0) continue;
                            mx = std::max(mx, ++bank[(a * (long long)SE + ad) & 31]);
                        }
                        cyc += mx;
                    }
    };
    // check phase (wavefronts 1..): edge u of check i is CSR edge row_ptr[i] + u
    pass(m, 64, max_rw, [&](int i, int u) -> long long {
        return u < row_ptr[i + 1] - row_ptr[i] ? (long long)row_ptr[i] + u : -1;
    });
    // fault phase (every wavefront): edge u of fault j is the CSR edge col_edge[col_ptr[j] + u]
    pass(n, 0, max_cw, [&](int j, int u) -> long long {
        return u < col_ptr[j + 1] - col_ptr[j] ? (long long)col_edge[col_ptr[j] + u] : -1;
    });
    return cyc;
}

// The message stride (floats per slot) of S slots within `budget` bytes of LDS: the fewest modelled
// bank cycles among E .. E + 63 (the smallest stride on ties).  On the [[144,12,12]] code (432
// edges, 14 slots) the odd stride 433 models 2.8 and 2.6 cycles per half-wavefront access in the
// check and fault phases, the chosen 437 models 1.0 and 1.5, and BP ran 6 % faster; the stride a
// 64-bank model prefers ran slower than 437, which is why the model counts 32 banks.
int bp_msg_stride(const DevGraph &g, const int32_t *row_ptr, const int32_t *col_ptr, const int32_t *col_edge, int S,
                  size_t budget) {
    int best = bp_min_stride(g);
    if (S < 1) return best;
    long long best_cyc = -1;
    for (int SE = g.nnz; SE < g.nnz + 64; SE++) {
        if (bp_lds_bytes(g, S, SE) > budget) break;
        const long long c = bp_bank_cycles(row_ptr, col_ptr, col_edge, g.m, g.n, g.max_rw, g.max_cw, S, SE);
        if (best_cyc < 0 || c < best_cyc) { best_cyc = c; best = SE; }
    }
    return best;
}

template <int RW, int CW, bool REG, int LSDW, bool OVF>
static hipError_t launch_bp_t(const BpArgs &a, const FuseArgs &f, int grid, size_t lds, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)bp_lds_kernel<RW, CW, REG, LSDW, OVF>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((bp_lds_kernel<RW, CW, REG, LSDW, OVF>), dim3(grid), dim3(kBpThreads), lds, st, a, f);
    return hipGetLastError();
}

// Large graphs, fault-major message order.  The messages of fault j sit contiguously at its CSC
// positions col_ptr[j] .. col_ptr[j+1]; each thread keeps the graph structure it touches in
// registers for the kernel's lifetime -- for each of its FPT faults the index, CSC start, degree
// and prior, and for its check row (needs m <= NT) the CSC positions of the row's edges -- so the
// iteration loop reads no graph tables (only the row indices of faults whose hard decision is 1,
// for the parity words).  Thread t takes the faults at positions t + k*NT of the code's fault
// order and the check at position t of its check order (both by decreasing weight), so almost
// every wavefront's 64 faults, or checks, have one weight: such a wavefront runs its loops over
// the messages to that weight with scalar branches only, the few mixed ones with a per-lane test
// on each message.  Same arithmetic, in the same order, as bp_graph_kernel; which thread computes
// a fault or a check changes no result.
template <int MAXRW, int MAXCW, int FPT>
__global__ __launch_bounds__(kBpGraphThreads) void bp_graph2_kernel(BpArgs args) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = threadIdx.x, NT = blockDim.x;
    const int m = args.g.m, n = args.g.n, MW = args.g.msg_words;
    const int PW = (m + 31) / 32;
    float *msg = (float *)smem;  // the layout of bp_graph2_layout: fault entry u at its word + 64 u
    float *Lv = msg + MW;
    uint32_t *synw = (uint32_t *)(Lv + n);
    uint32_t *parw = synw + PW;
    int *ctl = (int *)(parw + PW);
    const int32_t *row_idx = args.g.row_idx;
    const float alpha = args.alpha;
    const int T = args.max_iter;
    const int lane = t & 63, wave = t >> 6;

    // fault record: LDS word of its first message (15 bits) | fault (14 bits) << 15 | degree (3 bits)
    // << 29; a record of degree 0 is no fault
    uint32_t fmeta[FPT];
    float flam[FPT];
#pragma unroll
    for (int k = 0; k < FPT; k++) {
        const int p = t + k * NT;
        uint32_t v = 0;
        float l = 0.f;
        if (p < n) {
            const int j = args.g.fault_order[p];
            v = (uint32_t)args.g.fault_msg[j] | ((uint32_t)j << 15) |
                ((uint32_t)(args.g.col_ptr[j + 1] - args.g.col_ptr[j]) << 29);
            l = args.lam[j];
        }
        fmeta[k] = v;
        flam[k] = l;
    }
    uint32_t rpos2[MAXRW / 2];  // LDS words of the row's messages in visiting order, two u16 per word
    const int ci = t < m ? args.g.check_order[t] : m;  // this thread's check (m: none)
    int rw = 0;
    if (ci < m) {
        const int e0 = args.g.row_ptr[ci];
        rw = args.g.row_ptr[ci + 1] - e0;
#pragma unroll
        for (int u = 0; u < MAXRW; u += 2) {
            const uint32_t lo = u < rw ? (uint32_t)args.g.row_msg[e0 + u] : 0u;
            const uint32_t hi = u + 1 < rw ? (uint32_t)args.g.row_msg[e0 + u + 1] : 0u;
            rpos2[u / 2] = lo | (hi << 16);
        }
    }

    for (;;) {
        if (t == 0) ctl[0] = atomicAdd(args.next_shot, 1);
        __syncthreads();
        const int shot = ctl[0];
        if (shot >= args.B) break;
        const uint8_t *syn = args.syn + (size_t)shot * m;
        for (int i0 = wave * 64; i0 < m; i0 += NT) {
            const int i = i0 + lane;
            const uint64_t bits = __ballot(i < m && (syn[i] & 1));
            if (lane == 0) {
                synw[i0 >> 5] = (uint32_t)bits;
                if ((i0 >> 5) + 1 < PW) synw[(i0 >> 5) + 1] = (uint32_t)(bits >> 32);
            }
        }
        for (int w = t; w < PW; w += NT) parw[w] = 0u;
        for (int e = t; e < MW; e += NT) msg[e] = 0.f;  // r = 0: the first fault phase sets q = lambda
        __syncthreads();
        int it = 0;
        bool conv = false;
        for (;;) {
            // fault phase
            // one fault's update; CWU: the wavefront's common degree (a run-time but wave-uniform
            // bound, scalar branches only) or, for a mixed wavefront, the lane's own degree
            auto fault_update = [&](int k, auto Uni) -> float {
                constexpr bool UNI = decltype(Uni)::value;
                const int c0 = (int)(fmeta[k] & 0x7fffu), cw = (int)(fmeta[k] >> 29);
                const int cwb = UNI ? __builtin_amdgcn_readfirstlane(cw) : cw;
                float r[MAXCW];
#pragma unroll
                for (int u = 0; u < MAXCW; u++) r[u] = u < cwb ? msg[c0 + 64 * u] : 0.f;
                float pre[MAXCW + 1];
                pre[0] = flam[k];
#pragma unroll
                for (int u = 0; u < MAXCW; u++) pre[u + 1] = pre[u] + r[u];
                float suf = 0.f;
#pragma unroll
                for (int u = MAXCW - 1; u >= 0; u--) {
                    if (u < cwb) {
                        msg[c0 + 64 * u] = clampf(pre[u] + suf);
                        suf += r[u];
                    }
                }
                return clampf(pre[MAXCW]);
            };
            // a uniform wavefront's degree as a compile-time constant: no branches in the loops
            auto fault_fixed = [&](int k, auto Dc) -> float {
                constexpr int D = decltype(Dc)::value;
                const int c0 = (int)(fmeta[k] & 0x7fffu);
                float r[D];
#pragma unroll
                for (int u = 0; u < D; u++) r[u] = msg[c0 + 64 * u];
                float pre[D + 1];
                pre[0] = flam[k];
#pragma unroll
                for (int u = 0; u < D; u++) pre[u + 1] = pre[u] + r[u];
                float suf = 0.f;
#pragma unroll
                for (int u = D - 1; u >= 0; u--) {
                    msg[c0 + 64 * u] = clampf(pre[u] + suf);
                    suf += r[u];
                }
                // the remaining MAXCW - D terms of the general form add +0 to pre[D]
                float last = pre[D];
#pragma unroll
                for (int u = D; u < MAXCW; u++) last = last + 0.f;
                return clampf(last);
            };
#pragma unroll
            for (int k = 0; k < FPT; k++) {
                const int cw = (int)(fmeta[k] >> 29);
                const int cwk = __builtin_amdgcn_readfirstlane(cw);
                const bool uni = __ballot(cw != cwk) == 0;
                float Lt = 0.f;
                if (uni) {
                    switch (cwk) {
                        case 0: break;
                        case 1: Lt = fault_fixed(k, std::integral_constant<int, 1>{}); break;
                        case 2: Lt = fault_fixed(k, std::integral_constant<int, 2>{}); break;
                        case 3: Lt = fault_fixed(k, std::integral_constant<int, 3>{}); break;
                        case 4: Lt = fault_fixed(k, std::integral_constant<int, 4>{}); break;
                        default: Lt = fault_update(k, std::true_type{}); break;
                    }
                } else if (cw > 0) {
                    Lt = fault_update(k, std::false_type{});
                }
                if (cw > 0) {
                    const int j = (int)((fmeta[k] >> 15) & 0x3fffu);
                    Lv[j] = Lt;
                    if (Lt < 0.f) {
                        const int cs = args.g.col_ptr[j];  // the fault's CSC entries
                        for (int u = 0; u < cw; u++) {
                            const int i = row_idx[cs + u];
                            atomicXor(parw + (i >> 5), 1u << (i & 31));
                        }
                    }
                }
            }
            __syncthreads();
            // syndrome test of the hard decision after iteration it (it >= 1)
            if (wave == 0) {
                bool ok = true;
                for (int w = lane; w < PW; w += 64) {
                    ok &= parw[w] == synw[w];
                    parw[w] = 0u;
                }
                const bool all = __ballot(!ok) == 0;
                if (lane == 0) ctl[1] = all ? 1 : 0;
            }
            __syncthreads();
            const bool sat = ctl[1] != 0;
            conv = it >= 1 && sat;
            if ((args.early_exit && conv) || it >= T) break;
            it++;
            // check phase: thread t owns check t; two passes over the row's messages (minima and
            // sign, then the updates) instead of holding them in registers
            auto check_update = [&](auto Uni) {
                constexpr bool UNI = decltype(Uni)::value;
                const int rwb = UNI ? __builtin_amdgcn_readfirstlane(rw) : rw;
                const uint32_t sb = (synw[ci >> 5] >> (ci & 31)) & 1u;
                uint32_t sg = sb << 31;
                float mn1 = INFINITY, mn2 = INFINITY;
#pragma unroll
                for (int u = 0; u < MAXRW; u++) {
                    if (u < rwb) {
                        const float q = msg[(rpos2[u / 2] >> (16 * (u & 1))) & 0xffffu];
                        sg ^= __float_as_uint(q);
                        const float a = fabsf(q);
                        mn2 = __builtin_amdgcn_fmed3f(mn1, mn2, a);
                        mn1 = fminf(mn1, a);
                    }
                }
                const float m1 = alpha * mn1, m2 = alpha * mn2;
#pragma unroll
                for (int u = 0; u < MAXRW; u++) {
                    if (u < rwb) {
                        const int p = (rpos2[u / 2] >> (16 * (u & 1))) & 0xffffu;
                        const float q = msg[p];
                        const float mag = (fabsf(q) == mn1) ? m2 : m1;
                        const uint32_t sgn = (sg ^ __float_as_uint(q)) & 0x80000000u;
                        msg[p] = __uint_as_float(__float_as_uint(mag) | sgn);
                    }
                }
            };
            {
                const bool uni = __ballot(rw != __builtin_amdgcn_readfirstlane(rw)) == 0;
                if (uni) {
                    if (__builtin_amdgcn_readfirstlane(rw) > 0) check_update(std::true_type{});
                } else if (rw > 0) {
                    check_update(std::false_type{});
                }
            }
            __syncthreads();
        }
        // outputs
        const size_t row = (size_t)shot * n;
        for (int j = t; j < n; j += NT) {
            const float Lj = Lv[j];
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
            if (args.lsd_flag) args.lsd_flag[shot] = conv ? 0 : 1;
        }
        __syncthreads();
    }
}

size_t bp_graph_lds_bytes(const DevGraph &g) {
    // messages (the CSC order of bp_graph_kernel, or the padded layout of bp_graph2_kernel),
    // posteriors, syndrome and parity words, control words
    const size_t PW = ((size_t)g.m + 31) / 32;
    const size_t words = std::max<size_t>((size_t)g.nnz, (size_t)std::max(g.msg_words, 0));
    return align16(sizeof(float) * (words + g.n) + sizeof(uint32_t) * 2 * PW + sizeof(int) * 4);
}

// Message layout of bp_graph2_kernel, chosen so that both phases' LDS accesses spread over the
// banks (gfx950 serves a wavefront's 32-bit LDS accesses as two halves of 32 lanes over 32 banks
// of 4 bytes).  Fault phase: lane l of the wavefront that takes positions 64 g .. 64 g + 63 of the
// weight order reads entry u of its fault at word base_g + 64 u + l, so the 32 lanes of a half
// read 32 consecutive words (base_g: 64 times the largest weight of the groups before).  Check
// phase: thread t takes check t of the check order and visits its edges in an order of its own
// (min-sum's minima and sign product do not depend on the order); within each half of a
// wavefront, the checks' picks at each visit step form a maximum matching between the checks and
// the banks of their edges not yet visited (augmenting paths; edges tried in order of their bank's
// count of unvisited edges in the half, most first).  On the 936 x 8800 detector error model this
// models 1.0 instead of 3.2 cycles per half-wavefront access in the fault phase (the CSC order
// follows fault indices, not the weight order the lanes follow) and 1.6 instead of 3.4 in the
// check phase (2.0 with a greedy pick per check; the banks' loads bound it below by about 1.4),
// for 24,832 words instead of 24,643.
int bp_graph2_layout(int m, int n, int nnz, const int32_t *row_ptr, const int32_t *col_ptr, const int32_t *row_edge,
                     const int32_t *fault_order, const int32_t *check_order, std::vector<int32_t> &fault_msg,
                     std::vector<uint16_t> &row_msg) {
    if (m > kBpGraphThreads || n <= 0 || nnz <= 0) return -1;
    fault_msg.assign((size_t)n, 0);
    std::vector<int32_t> csc_msg((size_t)nnz, 0);
    long long base = 0;
    for (int g0 = 0; g0 < n; g0 += 64) {
        const int g1 = std::min(n, g0 + 64);
        int maxw = 0;
        for (int p = g0; p < g1; p++) {
            const int j = fault_order[p];
            maxw = std::max(maxw, col_ptr[j + 1] - col_ptr[j]);
        }
        for (int p = g0; p < g1; p++) {
            const int j = fault_order[p], l = p - g0;
            fault_msg[j] = (int32_t)(base + l);
            for (int u = 0; u < col_ptr[j + 1] - col_ptr[j]; u++) csc_msg[col_ptr[j] + u] = (int32_t)(base + 64 * u + l);
        }
        base += 64ll * maxw;
    }
    if (base >= 32768) return -1;  // the packed fault record holds 15 bits
    row_msg.assign((size_t)nnz, 0);
    for (int h0 = 0; h0 < m; h0 += 32) {
        const int h1 = std::min(m, h0 + 32);
        int hmax = 0;
        for (int p = h0; p < h1; p++) hmax = std::max(hmax, row_ptr[check_order[p] + 1] - row_ptr[check_order[p]]);
        // edges of each check not yet visited (CSR edge ids), kept in ascending order
        std::vector<std::vector<int>> left((size_t)(h1 - h0));
        for (int p = h0; p < h1; p++) {
            const int i = check_order[p];
            for (int e = row_ptr[i]; e < row_ptr[i + 1]; e++) left[(size_t)(p - h0)].push_back(e);
        }
        for (int u = 0; u < hmax; u++) {
            // this step's picks: a maximum matching of the half's checks to the 32 banks (each
            // check one unvisited edge, each bank one check), each check trying its edges in order
            // of their bank's count of unvisited edges in the half (most first), then edge id;
            // a check left unmatched takes an edge in the bank fewest picks use
            int load[32] = {0};
            for (const auto &lp : left)
                for (int e : lp) load[csc_msg[row_edge[e]] & 31]++;
            std::vector<std::vector<int>> cand(left.size());
            for (size_t q = 0; q < left.size(); q++) {
                cand[q] = left[q];
                std::stable_sort(cand[q].begin(), cand[q].end(), [&](int x, int y) {
                    return load[csc_msg[row_edge[x]] & 31] > load[csc_msg[row_edge[y]] & 31];
                });
            }
            int owner[32], owner_edge[32];
            std::fill(owner, owner + 32, -1);
            std::fill(owner_edge, owner_edge + 32, -1);
            bool seen[32];
            std::function<bool(int)> augment = [&](int q) -> bool {
                for (int e : cand[(size_t)q]) {
                    const int b = csc_msg[row_edge[e]] & 31;
                    if (seen[b]) continue;
                    seen[b] = true;
                    if (owner[b] < 0 || augment(owner[b])) {
                        owner[b] = q;
                        owner_edge[b] = e;
                        return true;
                    }
                }
                return false;
            };
            for (size_t q = 0; q < left.size(); q++) {
                if (left[q].empty()) continue;
                std::fill(seen, seen + 32, false);
                augment((int)q);
            }
            std::vector<int> pick(left.size(), -1);
            int cnt[32] = {0};
            for (int b = 0; b < 32; b++)
                if (owner[b] >= 0) {
                    pick[(size_t)owner[b]] = owner_edge[b];
                    cnt[b]++;
                }
            for (size_t q = 0; q < left.size(); q++) {
                if (left[q].empty() || pick[q] >= 0) continue;
                int best = left[q][0];
                for (int e : left[q])
                    if (cnt[csc_msg[row_edge[e]] & 31] < cnt[csc_msg[row_edge[best]] & 31]) best = e;
                pick[q] = best;
                cnt[csc_msg[row_edge[best]] & 31]++;
            }
            for (size_t q = 0; q < left.size(); q++) {
                if (pick[q] < 0) continue;
                row_msg[(size_t)row_ptr[check_order[h0 + (int)q]] + u] = (uint16_t)csc_msg[row_edge[pick[q]]];
                left[q].erase(std::find(left[q].begin(), left[q].end(), pick[q]));
            }
        }
    }
    return (int)base;
}

template <int RW, int CW>
static hipError_t launch_bp_graph_t(const BpArgs &a, int grid, size_t lds, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)bp_graph_kernel<RW, CW>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((bp_graph_kernel<RW, CW>), dim3(grid), dim3(kBpGraphThreads), lds, st, a);
    return hipGetLastError();
}

template <int RW, int CW, int FPT>
static hipError_t launch_bp_graph2_t(const BpArgs &a, int grid, size_t lds, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)bp_graph2_kernel<RW, CW, FPT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((bp_graph2_kernel<RW, CW, FPT>), dim3(grid), dim3(kBpGraphThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_bp_graph(const BpArgs &a, int grid, hipStream_t st) {
    const size_t lds = bp_graph_lds_bytes(a.g);
    // register-resident structure: checks <= threads, row weight <= 32, column weight <= 8, u16
    // CSC positions, at most 9 faults per thread (the 936 x 8800 detector error model)
    const DevGraph &g = a.g;
    // the packed fault record needs nnz < 2^15, n < 2^14, column weight <= 7
    if (g.m <= kBpGraphThreads && g.max_rw <= 32 && g.max_cw <= 7 && g.nnz < 32768 && g.n <= 9 * kBpGraphThreads &&
        g.n < 16384 && g.fault_order && g.check_order && g.fault_msg && g.row_msg && g.msg_words > 0 &&
        g.msg_words < 32768)
        return launch_bp_graph2_t<32, 8, 9>(a, grid, lds, st);
    if (a.g.max_rw <= 8 && a.g.max_cw <= 4) return launch_bp_graph_t<8, 4>(a, grid, lds, st);
    if (a.g.max_rw <= 16 && a.g.max_cw <= 8) return launch_bp_graph_t<16, 8>(a, grid, lds, st);
    return launch_bp_graph_t<kMaxRowWeight, kMaxColWeight>(a, grid, lds, st);
}

template <int LSDW, bool OVF = false>
static hipError_t launch_bp_w(const BpArgs &a, const FuseArgs &f, int grid, size_t lds, hipStream_t st) {
    const DevGraph &g = a.g;
    if (bp_regular63(g)) return launch_bp_t<6, 3, true, LSDW, OVF>(a, f, grid, lds, st);
    if (g.max_rw <= 8 && g.max_cw <= 4) return launch_bp_t<8, 4, false, LSDW, OVF>(a, f, grid, lds, st);
    if (g.max_rw <= 16 && g.max_cw <= 8) return launch_bp_t<16, 8, false, LSDW, OVF>(a, f, grid, lds, st);
    return launch_bp_t<kMaxRowWeight, kMaxColWeight, false, LSDW, OVF>(a, f, grid, lds, st);
}

hipError_t launch_bp(const BpArgs &a, int grid, hipStream_t st) {
    FuseArgs f;
    memset(&f, 0, sizeof(f));
    return launch_bp_w<0>(a, f, grid, bp_lds_bytes(a.g, a.S, a.SE), st);
}

hipError_t launch_bp_fused(const BpArgs &a, const FuseArgs &f, int W, int grid, hipStream_t st) {
    const size_t lds = std::max(bp_lds_bytes(a.g, a.S, a.SE), (size_t)f.lsd_bytes);
    if (f.lsd.ovf_list && a.g.m > 64 * W) {
        switch (W) {
            case 1: return launch_bp_w<1, true>(a, f, grid, lds, st);
            case 2: return launch_bp_w<2, true>(a, f, grid, lds, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (W) {
        case 1: return launch_bp_w<1>(a, f, grid, lds, st);
        case 2: return launch_bp_w<2>(a, f, grid, lds, st);
        default: return hipErrorInvalidValue;  // W = 4 would double the registers of the BP part
    }
}

namespace {
__global__ void fill_kernel(int *p, int count, int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// Two fills in one launch (one launch and one gap less in front of a decode).
__global__ void fill2_kernel(int *p1, int n1, int v1, int *p2, int n2, int v2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n1) p1[i] = v1;
    else if (i - n1 < n2) p2[i - n1] = v2;
}

}  // namespace



hipError_t launch_fill(int *p, int count, int value, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3((count + 255) / 256), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

hipError_t launch_zero(int *p, int count, hipStream_t st) { return launch_fill(p, count, 0, st); }

hipError_t launch_fill2(int *p1, int n1, int v1, int *p2, int n2, int v2, hipStream_t st) {
    const int total = std::max(n1, 0) + std::max(n2, 0);
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill2_kernel, dim3((total + 255) / 256), dim3(256), 0, st, p1, std::max(n1, 0), v1, p2,
                       std::max(n2, 0), v2);
    return hipGetLastError();
}

}  // namespace qlsd
