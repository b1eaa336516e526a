// Internal declarations shared by the HIP kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/qlsd.h"

namespace qlsd {

// Device copy of H: CSR (checks -> faults) and CSC (faults -> checks); edge id = CSR position.
struct DevGraph {
    int m, n, nnz;
    int max_rw, max_cw;
    int min_rw, min_cw;
    const int32_t *row_ptr, *col_idx;   // m+1, nnz
    const int32_t *col_ptr, *row_idx;   // n+1, nnz
    const int32_t *col_edge;            // nnz: CSR edge id of each CSC entry
    const int32_t *row_edge;            // nnz: CSC position of each CSR edge (inverse of col_edge)
    const int32_t *fault_order;         // n: faults by decreasing column weight, ties by index
    const int32_t *check_order;         // m: checks by decreasing row weight, ties by index
    // message layout of the large-graph BP kernel (bp_graph2_layout; null / 0 when not built):
    const int32_t *fault_msg;           // n: LDS word of each fault's first message (entry u: + 64 u)
    const uint16_t *row_msg;            // nnz: per check, in CSR slots, the LDS words of its messages
                                        // in the order the check phase visits them
    int msg_words;                      // LDS words the layout spans
};

// Arguments of the BP kernel (messages resident in LDS, persistent slots).
struct BpArgs {
    DevGraph g;
    const float *lam;          // n, prior LLRs (float32)
    const uint8_t *syn;        // B x m
    int B;
    int max_iter;
    float alpha;
    int early_exit;
    int S;                     // shot slots per workgroup
    int SE;                    // message stride per slot (floats, >= nnz; bp_msg_stride)
    int *next_shot;            // queue head (zeroed before launch)
    uint8_t *corr;             // B x n: hard decision of the last iteration (nullable)
    float *llr_out;            // B x n: posterior LLRs of every shot (nullable)
    float *llr_lsd;            // B x n: posterior LLRs of shots that did not converge (nullable)
    uint8_t *lsd_flag;         // B: 1 iff the shot did not converge and goes to LSD (nullable)
    qlsd_shot_info *info;      // B (nullable)
};

// Arguments of the LSD kernel (one wavefront per shot).
struct LsdArgs {
    DevGraph g;
    const uint8_t *syn;        // B x m
    const float *llr;          // B x n soft information
    const int *list;           // shots to decode (nullable: shots 0..count-1)
    const int *list_count;     // device count when list != nullptr
    int count;                 // count when list == nullptr
    int *next_item;            // work counter (zeroed before launch)
    uint8_t *corr;             // B x n
    qlsd_shot_info *info;      // B (nullable)
    int bp_iters;              // info.bp_iters of every shot decoded: BP's budget when BP ran first
                               // (a shot BP leaves unsolved ran all of it), 0 otherwise
    int keys_in_lds;
    int graph_in_lds;          // H staged as u16 CSR/CSC in LDS once per workgroup
    int mu;                    // LSD order (0 = LSD-0): extra growth rounds, and the OSD-E order
    int cs_order;              // > 0: local reprocessing is OSD-CS of this order instead of OSD-E
    const int64_t *omega;      // n: integer fault weights for the order-mu search (mu > 0)
    int wave_bytes;            // LDS bytes per wavefront
    int coherent_llr;          // llr rows written during this kernel by other workgroups: read them
                               // with device-scope atomics
    int skip_done;             // list entries < 0 were decoded already (after the fused kernel)
    int *done_count;           // with skip_done: how many were (nullable); all done -> no work
    int *ovf_list;             // nullable: shots whose clusters outgrew the kernel's capacity are
    int *ovf_count;            //   appended here for the next overflow kernel (max_batch entries)
    qlsd_cluster_stats *cstats;  // B (nullable): per-shot statistics of the final clusters
    int cluster_batched;       // W = 4 kernel: reduce the round's columns batched across clusters
};

// BP with LSD folded in (plain decode with slot BP): a workgroup whose slots have drained turns
// its wavefronts to LSD on shots that BP workgroups have published as unsolved.  lsd.list is the
// published list (every entry -1 before launch), lsd.list_count (tail) its reservation count and
// lsd.next_item a ticket counter: a wavefront takes ticket h, waits for entry h, decodes it and
// marks it done (~shot).  It leaves when entry h will never exist or after a bounded wait, so
// the stand-alone LSD kernel launched afterwards (skip_done) decodes every entry not marked done.
struct FuseArgs {
    LsdArgs lsd;
    int *list_w;               // writable alias of lsd.list
    int *tail;                 // == lsd.list_count
    int *bp_done;              // BP workgroups finished
    int *lsd_done;             // shots decoded by the fused kernel (== lsd.done_count)
    int lsd_waves;             // wavefronts per workgroup that run LSD (LDS permitting)
    int lsd_bytes;             // dynamic LDS the kernel needs (>= the BP carve)
};

// LDS carve sizes (bytes) shared by host (launch config) and device.
size_t bp_lds_bytes(const DevGraph &g, int S, int SE);
// the slot kernel's message stride: the smallest (odd) one, and the one a model of the LDS banks
// picks for S slots within budget bytes (host copies of the CSR row pointers and the CSC layout)
int bp_min_stride(const DevGraph &g);
int bp_msg_stride(const DevGraph &g, const int32_t *row_ptr, const int32_t *col_ptr, const int32_t *col_edge, int S,
                  size_t budget);
size_t bp_graph_lds_bytes(const DevGraph &g);
// Builds the large-graph kernel's message layout on the host (see qlsd_bp.hip); returns the
// LDS words it spans, or -1 when the kernel's limits rule it out.
int bp_graph2_layout(int m, int n, int nnz, const int32_t *row_ptr, const int32_t *col_ptr, const int32_t *row_edge,
                     const int32_t *fault_order, const int32_t *check_order, std::vector<int32_t> &fault_msg,
                     std::vector<uint16_t> &row_msg);
// with_mu: the decoder runs LSD-mu (order > 0) and needs the LSD-mu arrays
size_t lsd_wave_bytes(const DevGraph &g, int W, bool keys_in_lds, bool with_mu);
size_t lsd_total_lds(const DevGraph &g, int W, bool keys_in_lds, bool graph_in_lds, bool with_mu);

hipError_t launch_zero(int *p, int count, hipStream_t st);
hipError_t launch_fill(int *p, int count, int value, hipStream_t st);
hipError_t launch_fill2(int *p1, int n1, int v1, int *p2, int n2, int v2, hipStream_t st);
hipError_t launch_bp(const BpArgs &a, int grid, hipStream_t st);        // S slots per workgroup
hipError_t launch_bp_fused(const BpArgs &a, const FuseArgs &f, int W, int grid, hipStream_t st);
size_t bp_tables_bytes(const DevGraph &g);  // graph tables (u16 copies of H) at the start of the BP LDS block
hipError_t launch_bp_graph(const BpArgs &a, int grid, hipStream_t st);  // one workgroup per shot
hipError_t launch_lsd(const LsdArgs &a, int W, int grid, hipStream_t st);
// Wide LSD: one wavefront per workgroup, local-row capacity kWideRows, the Gauss-Jordan basis in
// ws (grid * lsd_wide_ws_words() words); decodes the shots listed in a.list / *a.list_count.
constexpr int kWideW = 16;
constexpr int kWideRows = 64 * kWideW;
constexpr int kWideDependent = 4096;  // LSD-mu: dependent clustered columns the overflow kernels can list
size_t lsd_wide_ws_words();                 // per workgroup
size_t lsd_wide_lds(const DevGraph &g, bool keys_in_lds, bool with_mu);
hipError_t launch_lsd_wide(const LsdArgs &a, uint64_t *ws, int grid, hipStream_t st);
// Mid LSD: as the wide kernel with kMidRows local rows and the basis in LDS (no workspace); shots
// that outgrow it are appended to a.ovf_list / a.ovf_count (when set) for the wide kernel.
constexpr int kMidW = 8;
constexpr int kMidRows = 64 * kMidW;
size_t lsd_mid_lds(const DevGraph &g, bool keys_in_lds, bool with_mu);
hipError_t launch_lsd_mid(const LsdArgs &a, int grid, hipStream_t st);
hipError_t launch_compact(const uint8_t *flag, int B, int *list, int *count, hipStream_t st);

hipError_t launch_error_clusters(const DevGraph &g, const uint8_t *e, int B, qlsd_cluster_stats *out, hipStream_t st);

// Global OSD-0 (one wavefront per shot; qlsd_osd.hip).
struct OsdArgs {
    DevGraph g;
    const uint8_t *syn;        // B x m
    const float *llr;          // B x n soft information
    const int *list;           // shots to decode (nullable: shots 0..count-1)
    const int *list_count;
    int count;
    int *next_item;            // work counter (zeroed before launch)
    uint8_t *corr;             // B x n
    qlsd_shot_info *info;      // B (nullable)
    int bp_iters;
    int P;                     // sort length: a power of two >= n
    int wave_bytes;            // LDS per wavefront (osd0_wave_bytes)
    uint64_t *ws;              // W = kWideW: grid * 2 * W * W * 64 words of basis
    int cs_order;              // 0: OSD-0; w in [1, kOsdCsMaxOrder]: global OSD-CS of order w (W <= 4)
    const int64_t *omega;      // n integer weights (OSD-CS)
};
constexpr int kOsdMaxSort = 4096;  // OSD-0 sorts n <= 4096 keys in LDS
constexpr int kOsdCsMaxOrder = 12;
// LDS of global OSD-CS per wavefront, after the OSD-0 block: pivot weights, the pivot-part change
// and weight of the first w dependent columns, the dependent columns in key order
struct OsdCsLds {
    int64_t *wq;      // 64 W
    uint64_t *zk;     // kOsdCsMaxOrder * W
    int64_t *tw;      // kOsdCsMaxOrder
    int32_t *dep;     // n
};
__host__ __device__ inline size_t osd0_wave_bytes_w(int n, int W, int P, bool cs) {
    size_t b = ((size_t)P * 8 + (size_t)64 * W * 4 + (size_t)((n + 31) / 32) * 4 + 15) & ~(size_t)15;
    if (cs) b += (8 * ((size_t)64 * W + (size_t)kOsdCsMaxOrder * W + kOsdCsMaxOrder) + 4 * (size_t)n + 15) & ~(size_t)15;
    return b;
}
size_t osd0_wave_bytes(const DevGraph &g, int W, int P, bool cs);
hipError_t launch_osd0(const OsdArgs &a, int W, int grid, hipStream_t st);  // W in {1, 2, 4, kWideW}

// Host helpers shared by the ABI files.
void set_last_error(const char *fmt, ...);
int code_rows(qlsd_code c);
int code_cols(qlsd_code c);
size_t decoder_device_bytes(qlsd_decoder d);  // workspace allocated by qlsd_decoder_create
DevGraph code_graph(qlsd_code c);
size_t net_lds_bytes(const DevGraph &g, bool train);
void net_graph_dims(const struct qlsd_net_s *net, int *m, int *n);
size_t net_infer_workspace_bytes(const struct qlsd_net_s *net);  // 0 for LDS-resident inference
hipError_t net_refine_listed(struct qlsd_net_s *net, const float *lam, const uint8_t *syn, float *llr,
                             const int *list, const int *list_count, int max_count, unsigned char *ws,
                             hipStream_t st);

constexpr int kBpThreads = 256;
constexpr int kBpGraphThreads = 1024;
constexpr int kLsdThreads = 256;   // 4 wavefronts, each decodes its own shots
constexpr int kMaxRowWeight = 32;  // BP register arrays
constexpr int kMaxColWeight = 16;

}  // namespace qlsd
