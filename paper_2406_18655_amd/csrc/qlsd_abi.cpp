// C ABI of libqlsd: argument checking, device set-up and launch sequencing.
// Every step of the decode runs in the HIP kernels of qlsd_bp.hip and qlsd_lsd.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/qlsd_net.h"
#include "qlsd_internal.h"

using namespace qlsd;

namespace {

thread_local char g_err[512] = "";

qlsd_status fail(qlsd_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

#define HIP_OK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(QLSD_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
hipError_t dev_copy(T **dst, const T *src, size_t count) {
    *dst = nullptr;
    hipError_t e = hipMalloc((void **)dst, sizeof(T) * std::max<size_t>(count, 1));
    if (e != hipSuccess) return e;
    if (count) e = hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice);
    return e;
}

constexpr size_t kStaticScratchBytes = (size_t)48 << 20;
constexpr int kStaticMaxDevices = 64;
constexpr int kStaticWideGrid = 8;  // wide-LSD workgroups (and bases) in the static scratch
std::mutex g_scratch_mu;
unsigned char *g_scratch_dev[kStaticMaxDevices];  // device address of `scratch`, per device

constexpr size_t kBpLdsBudget = 40 * 1024;  // four BP workgroups per CU
constexpr int kMaxSlots = 64;
constexpr size_t kLdsPerCu = 160 * 1024;

}  // namespace

// Scratch of qlsd_decode_static: one array per GPU the library runs on, held until the process
// ends.  Host code never passes `scratch` itself (on the host it is only a stand-in for the
// symbol): it uses the device address hipGetSymbolAddress returns on each device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct qlsd_code_s {
    int device;
    DevGraph g;
    int32_t *d_row_ptr, *d_col_idx, *d_col_ptr, *d_row_idx, *d_col_edge, *d_row_edge;
    int32_t *d_fault_order, *d_check_order;
    int32_t *d_fault_msg;  // message layout of the large-graph BP kernel (null when not built)
    uint16_t *d_row_msg;
    int min_rw;
    // host copies of the CSR row pointers and the CSC layout, for launch planning
    std::vector<int32_t> h_row_ptr, h_col_ptr, h_col_edge;
    // message strides already chosen for (slots, LDS budget): decoders of one code (serving
    // lanes) reuse them instead of re-running the model
    std::mutex stride_mu;
    std::vector<std::pair<std::pair<int, size_t>, int>> strides;
};

struct qlsd_decoder_s {
    qlsd_code code;
    qlsd_params params;
    int max_batch;
    float *d_lam;
    int64_t *d_omega;
    int *d_ctl;          // counters, one per 128-byte line (kCtl*): BP queue, LSD list length, LSD work
                         // counter (one-kernel path: tickets), BP workgroups done, work counter of the
                         // LSD launch after the one-kernel path, shots decoded inside it
    uint8_t *d_flag;     // max_batch: shot goes from BP to LSD
    int *d_list;         // max_batch: flagged shots, compacted
    float *d_llr;        // max_batch x n (LLRs handed from BP to LSD)
    int bp_slots, bp_grid;
    int bp_se;           // message stride per slot (bp_msg_stride)
    bool bp_graph;       // one workgroup per shot (large graphs) instead of S slots per workgroup
    int lsd_W, lsd_grid, lsd_wave_bytes, lsd_keys_in_lds, lsd_graph_in_lds;
    bool lsd_cb;         // cluster-batched column insertion (W = 4; qlsd_decoder_set_lsd_schedule)
    int num_cus;
    hipEvent_t ev[3];   // stage timing: before BP, between BP and LSD, after LSD
    bool timing;        // the events exist (QLSD_FLAG_STAGE_TIMING)
    bool timing_on;     // qlsd_decode records them (qlsd_decoder_set_stage_timing)
    qlsd_net net;       // optional refinement between BP and LSD
    unsigned char *d_netws;  // feature workspace of the refinement on large graphs (else nullptr)
    size_t netws_bytes;
    // shots whose clusters can outgrow the LSD kernel's 64 * lsd_W local rows (or, with LSD-mu,
    // its dependent-column list) are listed (ovf) and go on to the mid LSD kernel (512 local rows,
    // basis in LDS), and those that outgrow it to the wide LSD kernel (1024 rows, basis in device
    // memory); either tier is left out when it cannot be needed or does not fit in LDS
    bool ovf, mid, wide;
    int mid_grid, mid_keys_in_lds, wide_grid, wide_keys_in_lds;
    int *d_ovf_list;     // max_batch: shots the LSD kernel could not hold
    int *d_ovf2_list;    // max_batch (mid and wide): shots the mid kernel could not hold
    uint64_t *d_wide_ws; // wide_grid * lsd_wide_ws_words(): the wide kernel's Gauss-Jordan bases (also
                         // the global OSD-0 basis when m > 256)
    // global OSD-0 (qlsd_osd0, QLSD_FLAG_OSD0_POST): basis words per lane row, sort length
    int osd_W, osd_P, osd_wave_bytes;
    bool osd_ok;
    int osd_cs_wave_bytes;  // global OSD-CS (qlsd_osd_cs; QLSD_FLAG_OSD0_POST with osd_method 1)
    bool osd_cs_ok;
};

namespace qlsd {
// Decoder counters, each on its own 128-byte line: the one-kernel path polls the list counters
// while BP workgroups hit the queue counter, and atomics on a shared line would serialise.
constexpr int kCtlQueue = 0, kCtlList = 32, kCtlItem = 64, kCtlBpDone = 96, kCtlItem2 = 128, kCtlLsdDone = 160,
              kCtlOvf = 192, kCtlItemW = 224, kCtlOvf2 = 256, kCtlItemM = 288;
constexpr int kCtlWords = 320;
void set_last_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}
int code_rows(qlsd_code c) { return c->g.m; }
DevGraph code_graph(qlsd_code c) { return c->g; }
int code_cols(qlsd_code c) { return c->g.n; }
size_t decoder_device_bytes(qlsd_decoder d) {
    const size_t n = (size_t)d->code->g.n, B = (size_t)d->max_batch;
    return n * (sizeof(float) + sizeof(int64_t)) + kCtlWords * sizeof(int) + B * (1 + sizeof(int) + n * sizeof(float)) +
           d->netws_bytes + (d->d_ovf_list ? B * sizeof(int) : 0) + (d->d_ovf2_list ? B * sizeof(int) : 0) +
           (d->d_wide_ws ? (size_t)d->wide_grid * lsd_wide_ws_words() * sizeof(uint64_t) : 0);
}
}  // namespace qlsd

extern "C" {

// Overflow tiers of an LSD kernel with 64 W local rows (see the decoder fields) and their buffers,
// allocated when first needed; the wide kernel's workspace also serves global OSD-0 when m > 256.
// require: refuse (return false) when shots can overflow and no overflow kernel fits.  On false
// the decoder is left as it was.
static bool configure_overflow(qlsd_decoder d, int W, bool require) {
    const DevGraph &g = d->code->g;
    const bool with_mu = d->params.lsd_order > 0;
    const size_t lim = kLdsPerCu - 1024;
    const bool need = g.m > 64 * W || (with_mu && g.n > 64 * W);
    bool mid = false, mid_keys = false, wide = false, wide_keys = false;
    if (need) {
        // keys in LDS when they fit, else read from the LLR rows
        mid_keys = lsd_mid_lds(g, true, with_mu) <= lim;
        mid = mid_keys || lsd_mid_lds(g, false, with_mu) <= lim;
        if (!mid || g.m > kMidRows) {
            wide_keys = lsd_wide_lds(g, true, with_mu) <= lim;
            wide = wide_keys || lsd_wide_lds(g, false, with_mu) <= lim;
        }
    }
    const bool ovf = mid || wide;
    if (require && need && !ovf) return false;
    const bool wws = wide || d->osd_W == kWideW;
    const int wgrid = std::min(d->num_cus, 64);
    const size_t B = (size_t)d->max_batch;
    int *l1 = d->d_ovf_list, *l2 = d->d_ovf2_list;
    uint64_t *ws = d->d_wide_ws;
    bool ok = true;
    if (ok && ovf && !l1) ok = hipMalloc((void **)&l1, sizeof(int) * B) == hipSuccess;
    if (ok && mid && wide && !l2) ok = hipMalloc((void **)&l2, sizeof(int) * B) == hipSuccess;
    if (ok && wws && !ws) ok = hipMalloc((void **)&ws, sizeof(uint64_t) * (size_t)wgrid * lsd_wide_ws_words()) == hipSuccess;
    if (!ok) {
        if (l1 != d->d_ovf_list) hipFree(l1);
        if (l2 != d->d_ovf2_list) hipFree(l2);
        if (ws != d->d_wide_ws) hipFree(ws);
        return false;
    }
    if (ws != d->d_wide_ws) d->wide_grid = wgrid;
    d->d_ovf_list = l1;
    d->d_ovf2_list = l2;
    d->d_wide_ws = ws;
    d->ovf = ovf;
    d->mid = mid;
    d->mid_keys_in_lds = mid_keys;
    d->mid_grid = d->num_cus;
    d->wide = wide;
    d->wide_keys_in_lds = wide_keys;
    return true;
}

const char *qlsd_last_error(void) { return g_err; }

qlsd_status qlsd_code_create(int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                             const int32_t *col_idx, qlsd_code *out) {
    g_err[0] = 0;
    if (!out) return fail(QLSD_E_INVALID, "out is NULL");
    *out = nullptr;
    if (m < 1 || n < 1 || !row_ptr || (nnz > 0 && !col_idx))
        return fail(QLSD_E_INVALID, "bad shape m=%d n=%d or NULL arrays", m, n);
    if (nnz < 0 || nnz > (1ll << 30) || row_ptr[0] != 0 || row_ptr[m] != nnz)
        return fail(QLSD_E_INVALID, "row_ptr[0] must be 0 and row_ptr[m] == nnz");
    int max_rw = 0, min_rw = 1 << 30;
    for (int i = 0; i < m; i++) {
        const int a = row_ptr[i], b = row_ptr[i + 1];
        if (b < a) return fail(QLSD_E_INVALID, "row_ptr not monotone at row %d", i);
        max_rw = std::max(max_rw, b - a);
        min_rw = std::min(min_rw, b - a);
        for (int e = a; e < b; e++) {
            if (col_idx[e] < 0 || col_idx[e] >= n) return fail(QLSD_E_INVALID, "col_idx out of range at %d", e);
            if (e > a && col_idx[e] <= col_idx[e - 1])
                return fail(QLSD_E_INVALID, "columns of row %d not sorted/unique", i);
        }
    }
    std::vector<int32_t> col_ptr(n + 1, 0), row_idx(nnz), col_edge(nnz), row_edge(nnz), fill(n, 0);
    for (int64_t e = 0; e < nnz; e++) col_ptr[col_idx[e] + 1]++;
    int max_cw = 0, min_cw = 1 << 30;
    for (int j = 0; j < n; j++) {
        max_cw = std::max(max_cw, col_ptr[j + 1]);
        min_cw = std::min(min_cw, col_ptr[j + 1]);
        col_ptr[j + 1] += col_ptr[j];
    }
    for (int i = 0; i < m; i++)
        for (int e = row_ptr[i]; e < row_ptr[i + 1]; e++) {
            const int j = col_idx[e];
            const int k = col_ptr[j] + fill[j]++;
            row_idx[k] = i;
            col_edge[k] = e;
            row_edge[e] = k;
        }
    // faults by decreasing column weight and checks by decreasing row weight, ties by index
    // (stable counting sorts): kernels that give consecutive lanes consecutive entries then see
    // one weight in almost every wavefront
    auto order_by_weight = [](const int32_t *ptr, int count, int maxw) {
        std::vector<int32_t> ord(count);
        std::vector<int64_t> start((size_t)maxw + 2, 0);
        for (int x = 0; x < count; x++) start[(size_t)(maxw - (ptr[x + 1] - ptr[x])) + 1]++;
        for (int w = 1; w <= maxw + 1; w++) start[w] += start[w - 1];
        for (int x = 0; x < count; x++) ord[start[maxw - (ptr[x + 1] - ptr[x])]++] = x;
        return ord;
    };
    const std::vector<int32_t> fault_order = order_by_weight(col_ptr.data(), n, max_cw);
    const std::vector<int32_t> check_order = order_by_weight(row_ptr, m, max_rw);
    std::vector<int32_t> fault_msg;
    std::vector<uint16_t> row_msg;
    int msg_words = -1;
    try {
        msg_words = bp_graph2_layout(m, n, (int)nnz, row_ptr, col_ptr.data(), row_edge.data(), fault_order.data(),
                                     check_order.data(), fault_msg, row_msg);
    } catch (...) {
        return fail(QLSD_E_NOMEM, "host allocation failed");
    }
    qlsd_code c = new (std::nothrow) qlsd_code_s();
    if (!c) return fail(QLSD_E_NOMEM, "host allocation failed");
    HIP_OK(hipGetDevice(&c->device));
    hipError_t e1 = dev_copy(&c->d_row_ptr, row_ptr, (size_t)m + 1);
    hipError_t e2 = dev_copy(&c->d_col_idx, col_idx, (size_t)nnz);
    hipError_t e3 = dev_copy(&c->d_col_ptr, col_ptr.data(), (size_t)n + 1);
    hipError_t e4 = dev_copy(&c->d_row_idx, row_idx.data(), (size_t)nnz);
    hipError_t e5 = dev_copy(&c->d_col_edge, col_edge.data(), (size_t)nnz);
    if (e5 == hipSuccess) e5 = dev_copy(&c->d_row_edge, row_edge.data(), (size_t)nnz);
    if (e5 == hipSuccess) e5 = dev_copy(&c->d_fault_order, fault_order.data(), (size_t)n);
    if (e5 == hipSuccess) e5 = dev_copy(&c->d_check_order, check_order.data(), (size_t)m);
    if (e5 == hipSuccess && msg_words > 0) e5 = dev_copy(&c->d_fault_msg, fault_msg.data(), (size_t)n);
    if (e5 == hipSuccess && msg_words > 0) e5 = dev_copy(&c->d_row_msg, row_msg.data(), (size_t)nnz);
    if (e1 || e2 || e3 || e4 || e5) {
        qlsd_code_destroy(c);
        return fail(QLSD_E_NOMEM, "device allocation/copy of H failed");
    }
    c->g.m = m;
    c->g.n = n;
    c->g.nnz = (int)nnz;
    c->g.max_rw = max_rw;
    c->g.max_cw = max_cw;
    c->g.min_rw = min_rw;
    c->g.min_cw = min_cw;
    c->g.row_ptr = c->d_row_ptr;
    c->g.col_idx = c->d_col_idx;
    c->g.col_ptr = c->d_col_ptr;
    c->g.row_idx = c->d_row_idx;
    c->g.col_edge = c->d_col_edge;
    c->g.row_edge = c->d_row_edge;
    c->g.fault_order = c->d_fault_order;
    c->g.check_order = c->d_check_order;
    c->g.fault_msg = msg_words > 0 ? c->d_fault_msg : nullptr;
    c->g.row_msg = msg_words > 0 ? c->d_row_msg : nullptr;
    c->g.msg_words = std::max(msg_words, 0);
    c->min_rw = min_rw;
    try {
        c->h_row_ptr.assign(row_ptr, row_ptr + m + 1);
        c->h_col_ptr = col_ptr;
        c->h_col_edge = col_edge;
    } catch (...) {
        qlsd_code_destroy(c);
        return fail(QLSD_E_NOMEM, "host allocation failed");
    }
    *out = c;
    return QLSD_OK;
}

void qlsd_code_destroy(qlsd_code c) {
    if (!c) return;
    hipFree(c->d_row_ptr);
    hipFree(c->d_col_idx);
    hipFree(c->d_col_ptr);
    hipFree(c->d_row_idx);
    hipFree(c->d_row_edge);
    hipFree(c->d_col_edge);
    hipFree(c->d_fault_order);
    hipFree(c->d_check_order);
    hipFree(c->d_fault_msg);
    hipFree(c->d_row_msg);
    delete c;
}

// The slot kernel's message stride for S slots within budget bytes of LDS per workgroup.
static int bp_stride_for(qlsd_code c, int S, size_t budget) {
    std::lock_guard<std::mutex> lk(c->stride_mu);
    for (const auto &e : c->strides)
        if (e.first.first == S && e.first.second == budget) return e.second;
    const int se = bp_msg_stride(c->g, c->h_row_ptr.data(), c->h_col_ptr.data(), c->h_col_edge.data(), S, budget);
    try {
        c->strides.push_back({{S, budget}, se});
    } catch (...) {
    }
    return se;
}

qlsd_status qlsd_decoder_create(qlsd_code code, const qlsd_params *params, const double *priors,
                                int32_t max_batch, qlsd_decoder *out) {
    g_err[0] = 0;
    if (!out) return fail(QLSD_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!code || !params || !priors) return fail(QLSD_E_INVALID, "NULL code/params/priors");
    if (max_batch < 1) return fail(QLSD_E_BATCH, "max_batch must be >= 1");
    if (params->max_iter < 1 || params->max_iter > 30000) return fail(QLSD_E_INVALID, "max_iter out of range");
    if (!(params->ms_scaling > 0.f && params->ms_scaling <= 1.f)) return fail(QLSD_E_INVALID, "ms_scaling must be in (0,1]");
    if (params->osd_method != 0 && params->osd_method != 1)
        return fail(QLSD_E_UNSUPPORTED, "osd_method must be 0 (exhaustive) or 1 (combination sweep)");
    if (params->osd_method == 0 && (params->lsd_order < 0 || params->lsd_order > 12))
        return fail(QLSD_E_UNSUPPORTED, "lsd_order must be in [0, 12] with OSD-E");
    if (params->osd_method == 1 && (params->lsd_order < 0 || params->lsd_order > 4096 || params->osd_order < 1 ||
                                    params->osd_order > 12))
        return fail(QLSD_E_UNSUPPORTED, "OSD-CS needs lsd_order in [0, 4096] and osd_order in [1, 12]");
    const DevGraph &g = code->g;
    if (code->min_rw < 2) return fail(QLSD_E_INVALID, "BP needs every row weight >= 2");
    if (g.max_rw > kMaxRowWeight || g.max_cw > kMaxColWeight)
        return fail(QLSD_E_UNSUPPORTED, "row weight %d / column weight %d beyond %d / %d", g.max_rw, g.max_cw,
                    kMaxRowWeight, kMaxColWeight);
    std::vector<float> lam(g.n);
    std::vector<int64_t> omega(g.n);
    for (int j = 0; j < g.n; j++) {
        const double p = priors[j];
        if (!(p > 0.0 && p < 1.0)) return fail(QLSD_E_PRIOR, "prior %d = %g not in (0,1)", j, p);
        const double l = log((1.0 - p) / p);
        lam[j] = (float)l;
        omega[j] = (int64_t)llround(ldexp(l, 20));  // integer weight of the order-mu search
    }
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev != code->device) return fail(QLSD_E_INVALID, "code lives on device %d, current is %d", code->device, dev);
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));

    qlsd_decoder d = new (std::nothrow) qlsd_decoder_s();
    if (!d) return fail(QLSD_E_NOMEM, "host allocation failed");
    d->code = code;
    d->params = *params;
    d->max_batch = max_batch;
    d->num_cus = prop.multiProcessorCount;

    // BP: shot slots per workgroup.  Prefer 4 workgroups per CU (40 KB of LDS each) with at
    // least 12 slots; larger graphs take 2 (80 KB) or 1 (160 KB) workgroup per CU.
    int S = 0, wg_per_cu = 4;
    for (wg_per_cu = 4; wg_per_cu >= 1; wg_per_cu /= 2) {
        const size_t budget = kBpLdsBudget * (4 / wg_per_cu) - (wg_per_cu == 1 ? 1024 : 0);
        S = kMaxSlots;
        while (S > 0 && bp_lds_bytes(g, S, bp_min_stride(g)) > budget) S--;
        if (S >= 12 || (wg_per_cu == 1 && S >= 4)) break;
    }
    if (S >= 4 && g.n < 65535 && g.nnz < 65535) {
        d->bp_graph = false;
        d->bp_slots = S;
        d->bp_grid = std::max(1, wg_per_cu) * d->num_cus;
        const int tier = std::max(1, wg_per_cu);
        d->bp_se = bp_stride_for(code, S, kBpLdsBudget * (4 / tier) - (tier == 1 ? 1024 : 0));
    } else if (bp_graph_lds_bytes(g) <= kLdsPerCu - 1024) {
        // one workgroup per shot with the shot's messages in LDS
        d->bp_graph = true;
        d->bp_slots = 1;
        d->bp_grid = d->num_cus;
    } else {
        delete d;
        return fail(QLSD_E_UNSUPPORTED, "graph too large for LDS-resident BP (n=%d, nnz=%d)", g.n, g.nnz);
    }

    // LSD: local-row capacity 64*W
    int W = 1;
    while (64 * W < g.m && W < 4) W *= 2;
    if (params->lsd_order > 0) W = 4;  // extra growth steps: room for 256 clustered checks
    d->lsd_W = W;
    d->lsd_keys_in_lds = (size_t)g.n * 4 <= 16384;
    // the graph goes to LDS only with the keys (the LSD kernel then reads keys from LDS without a test)
    d->lsd_graph_in_lds = (2 * (size_t)g.nnz + g.m + g.n + 2) * 2 <= 24576 && g.n < 65536 && g.m < 65536 &&
                          d->lsd_keys_in_lds;
    const bool with_mu = params->lsd_order > 0;
    d->lsd_wave_bytes = (int)lsd_wave_bytes(g, W, d->lsd_keys_in_lds != 0, with_mu);
    if (lsd_total_lds(g, W, d->lsd_keys_in_lds != 0, d->lsd_graph_in_lds != 0, with_mu) > kLdsPerCu - 1024) {
        delete d;
        return fail(QLSD_E_UNSUPPORTED, "LSD workspace per wavefront too large");
    }
    d->lsd_grid = 8 * d->num_cus;
    // OSD-0: register basis for m <= 256, the wide (device-memory) basis up to 1024 rows, which
    // uses the wide LSD kernel's workspace (allocated below for every decoder with m > 256)
    d->osd_W = g.m <= 64 ? 1 : g.m <= 128 ? 2 : g.m <= 256 ? 4 : kWideW;
    d->osd_P = 1;
    while (d->osd_P < g.n) d->osd_P <<= 1;
    d->osd_wave_bytes = (int)osd0_wave_bytes(g, d->osd_W, d->osd_P, false);
    d->osd_ok = d->osd_P <= kOsdMaxSort && g.m <= kWideRows &&
                (size_t)d->osd_wave_bytes * (d->osd_W == kWideW ? 1 : 4) <= kLdsPerCu - 1024;
    d->osd_cs_wave_bytes = (int)osd0_wave_bytes(g, d->osd_W, d->osd_P, true);
    d->osd_cs_ok = d->osd_ok && d->osd_W != kWideW && (size_t)d->osd_cs_wave_bytes * 4 <= kLdsPerCu - 1024;
    if ((params->flags & QLSD_FLAG_OSD0_POST) && !d->osd_ok) {
        delete d;
        return fail(QLSD_E_UNSUPPORTED, "OSD-0 supports n <= %d and m <= %d (n=%d, m=%d)", kOsdMaxSort, kWideRows, g.n, g.m);
    }
    if ((params->flags & QLSD_FLAG_OSD0_POST) && params->osd_method == 1 && !d->osd_cs_ok) {
        delete d;
        return fail(QLSD_E_UNSUPPORTED, "global OSD-CS supports n <= %d and m <= 256 (n=%d, m=%d)", kOsdMaxSort, g.n, g.m);
    }
    d->lsd_cb = false;
    d->ovf = d->mid = d->wide = false;
    d->d_ovf_list = d->d_ovf2_list = nullptr;
    d->d_wide_ws = nullptr;
    d->wide_grid = d->mid_grid = 0;
    d->timing = (params->flags & QLSD_FLAG_STAGE_TIMING) != 0;
    d->timing_on = d->timing;
    for (int k = 0; k < 3; k++) d->ev[k] = nullptr;
    if (d->timing)
        for (int k = 0; k < 3; k++)
            if (hipEventCreate(&d->ev[k]) != hipSuccess) {
                qlsd_decoder_destroy(d);
                return fail(QLSD_E_DEVICE, "hipEventCreate failed");
            }

    hipError_t e1 = dev_copy(&d->d_lam, lam.data(), lam.size());
    if (e1 == hipSuccess) e1 = dev_copy(&d->d_omega, omega.data(), omega.size());
    hipError_t e2 = hipMalloc((void **)&d->d_ctl, sizeof(int) * kCtlWords);
    if (e2 == hipSuccess) e2 = hipMemset(d->d_ctl, 0, sizeof(int) * kCtlWords);
    hipError_t e3 = hipMalloc((void **)&d->d_flag, (size_t)max_batch);
    if (e3 == hipSuccess) e3 = hipMalloc((void **)&d->d_list, sizeof(int) * (size_t)max_batch);
    hipError_t e4 = hipMalloc((void **)&d->d_llr, sizeof(float) * (size_t)max_batch * g.n);
    // capacity of lsd_kernel: 64 W local rows (one per clustered detector, so never more than m)
    // and, with LSD-mu, 64 W dependent columns (never more than n); a graph too large for every
    // overflow kernel keeps the OVERFLOW status on such shots
    if (e4 == hipSuccess && !configure_overflow(d, W, false)) e4 = hipErrorOutOfMemory;
    if (e1 || e2 || e3 || e4) {
        qlsd_decoder_destroy(d);
        return fail(QLSD_E_NOMEM, "device workspace allocation failed (max_batch=%d)", max_batch);
    }
    *out = d;
    return QLSD_OK;
}

void qlsd_decoder_destroy(qlsd_decoder d) {
    if (!d) return;
    hipFree(d->d_lam);
    hipFree(d->d_omega);
    hipFree(d->d_ctl);
    hipFree(d->d_flag);
    hipFree(d->d_list);
    hipFree(d->d_llr);
    hipFree(d->d_netws);
    hipFree(d->d_ovf_list);
    hipFree(d->d_ovf2_list);
    hipFree(d->d_wide_ws);
    for (int k = 0; k < 3; k++)
        if (d->ev[k]) hipEventDestroy(d->ev[k]);
    delete d;
}

// Per-call device scratch of a decode: the decoder's own workspace (qlsd_decode and the other
// entry points) or a carve of the library's static scratch array (qlsd_decode_static).
struct Ws {
    int *ctl;           // kCtlWords counters
    uint8_t *flag;      // B: shot goes from BP to LSD
    int *list;          // B: shots for LSD
    float *llr;         // B x n: posteriors handed from BP to LSD
    int *ovf_list;      // B (decoders that can overflow): shots for the mid (else the wide) LSD kernel
    int *ovf2_list;     // B (mid and wide): shots for the wide LSD kernel
    uint64_t *wide_ws;  // wide_grid * lsd_wide_ws_words()
    int wide_grid;
};

static Ws decoder_ws(qlsd_decoder d) {
    return Ws{d->d_ctl, d->d_flag, d->d_list, d->d_llr, d->d_ovf_list, d->d_ovf2_list, d->d_wide_ws, d->wide_grid};
}

static BpArgs bp_args(qlsd_decoder d, const Ws &w, const uint8_t *syn, int B) {
    BpArgs a;
    memset(&a, 0, sizeof(a));
    a.g = d->code->g;
    a.lam = d->d_lam;
    a.syn = syn;
    a.B = B;
    a.max_iter = d->params.max_iter;
    a.alpha = d->params.ms_scaling;
    a.early_exit = (d->params.flags & QLSD_FLAG_NO_EARLY_EXIT) ? 0 : 1;
    a.S = d->bp_slots;
    a.SE = d->bp_se;
    a.next_shot = w.ctl + kCtlQueue;
    return a;
}

// Wavefronts per BP workgroup that can run LSD in the BP kernel's LDS block (past the graph
// tables); 0: BP and LSD run as separate kernels.  Only for LSD with up to 128 local rows (the
// one-kernel form then needs at most 128 VGPRs, i.e. 4 workgroups per CU, the BP default).
static int fuse_waves(qlsd_decoder d) {
    if (d->bp_graph || d->net || (d->params.flags & (QLSD_FLAG_SEPARATE_LSD | QLSD_FLAG_OSD0_POST))) return 0;
    if (d->lsd_W > 2 || d->params.lsd_order > 0 || !d->lsd_keys_in_lds || d->bp_grid > 4 * d->num_cus) return 0;
    const size_t avail = bp_lds_bytes(d->code->g, d->bp_slots, d->bp_se) - bp_tables_bytes(d->code->g);
    return (int)std::min<size_t>(4, avail / (size_t)d->lsd_wave_bytes);
}

static int bp_grid(qlsd_decoder d, int B) {
    const int need = (B + d->bp_slots - 1) / d->bp_slots;
    return std::max(1, std::min(d->bp_grid, need));
}

static hipError_t run_bp(qlsd_decoder d, const BpArgs &a, int B, hipStream_t s) {
    return d->bp_graph ? launch_bp_graph(a, bp_grid(d, B), s) : launch_bp(a, bp_grid(d, B), s);
}

static LsdArgs lsd_args(qlsd_decoder d, const Ws &w, const uint8_t *syn, const float *llr, uint8_t *corr,
                        qlsd_shot_info *info) {
    LsdArgs a;
    memset(&a, 0, sizeof(a));
    a.g = d->code->g;
    a.syn = syn;
    a.llr = llr;
    a.next_item = w.ctl + kCtlItem;
    a.corr = corr;
    a.info = info;
    a.keys_in_lds = d->lsd_keys_in_lds;
    a.graph_in_lds = d->lsd_graph_in_lds;
    a.mu = d->params.lsd_order;
    a.cs_order = d->params.osd_method == 1 ? d->params.osd_order : 0;
    a.omega = d->d_omega;
    a.wave_bytes = d->lsd_wave_bytes;
    a.cluster_batched = d->lsd_cb && d->lsd_W == 4;
    return a;
}

// LSD kernel arguments list overflowing shots for the overflow kernels (decoders that can overflow)
static void with_overflow_list(qlsd_decoder d, const Ws &w, LsdArgs &l) {
    if (!d->ovf) return;
    l.ovf_list = w.ovf_list;
    l.ovf_count = w.ctl + kCtlOvf;
}

// The overflow kernels over the shots the LSD kernel listed: the mid kernel, then the wide kernel
// over the shots the mid kernel listed (each exits at once when nothing was listed).
static hipError_t run_overflow(qlsd_decoder d, const Ws &ws, const uint8_t *syn, const float *llr, uint8_t *corr,
                               qlsd_shot_info *info, int bp_iters, hipStream_t s,
                               qlsd_cluster_stats *cstats = nullptr) {
    if (!d->ovf) return hipSuccess;
    if (d->mid) {
        LsdArgs x = lsd_args(d, ws, syn, llr, corr, info);
        x.list = ws.ovf_list;
        x.list_count = ws.ctl + kCtlOvf;
        x.next_item = ws.ctl + kCtlItemM;
        x.bp_iters = bp_iters;
        x.keys_in_lds = d->mid_keys_in_lds;
        x.graph_in_lds = 0;
        x.cstats = cstats;
        if (d->wide) {
            x.ovf_list = ws.ovf2_list;
            x.ovf_count = ws.ctl + kCtlOvf2;
        }
        const hipError_t e = launch_lsd_mid(x, d->mid_grid, s);
        if (e != hipSuccess || !d->wide) return e;
    }
    LsdArgs w = lsd_args(d, ws, syn, llr, corr, info);
    w.list = d->mid ? ws.ovf2_list : ws.ovf_list;
    w.list_count = ws.ctl + (d->mid ? kCtlOvf2 : kCtlOvf);
    w.next_item = ws.ctl + kCtlItemW;
    w.bp_iters = bp_iters;
    w.keys_in_lds = d->wide_keys_in_lds;
    w.graph_in_lds = 0;
    w.cstats = cstats;
    return launch_lsd_wide(w, ws.wide_ws, ws.wide_grid, s);
}

// Global OSD-0 (cs_order 0) or OSD-CS of order cs_order over the listed shots (list != nullptr)
// or shots 0..count-1.
static hipError_t run_osd0(qlsd_decoder d, const Ws &w, const uint8_t *syn, const float *llr, int count,
                           const int *list, const int *list_count, uint8_t *corr, qlsd_shot_info *info,
                           int bp_iters, hipStream_t s, int cs_order = 0) {
    OsdArgs a;
    memset(&a, 0, sizeof(a));
    a.g = d->code->g;
    a.syn = syn;
    a.llr = llr;
    a.list = list;
    a.list_count = list_count;
    a.count = count;
    a.next_item = w.ctl + kCtlItem;
    a.corr = corr;
    a.info = info;
    a.bp_iters = bp_iters;
    a.P = d->osd_P;
    a.wave_bytes = cs_order > 0 ? d->osd_cs_wave_bytes : d->osd_wave_bytes;
    a.ws = w.wide_ws;
    a.cs_order = cs_order;
    a.omega = d->d_omega;
    const int grid = d->osd_W == kWideW ? w.wide_grid : 8 * d->num_cus;
    return launch_osd0(a, d->osd_W, grid, s);
}

static qlsd_status check_call(qlsd_decoder d, const void *syn, int B, const void *out) {
    g_err[0] = 0;
    if (!d) return fail(QLSD_E_INVALID, "decoder is NULL");
    if (B < 0 || B > d->max_batch) return fail(QLSD_E_BATCH, "B=%d outside [0, %d]", B, d->max_batch);
    if (B > 0 && (!syn || !out)) return fail(QLSD_E_INVALID, "NULL syndromes or output");
    return QLSD_OK;
}

// BP then LSD on the per-call scratch w; timing: record the decoder's stage events.
static qlsd_status decode_with(qlsd_decoder d, const Ws &w, const uint8_t *syndromes, int B, uint8_t *corrections,
                               qlsd_shot_info *info, hipStream_t s, bool timing) {
    const int fw = fuse_waves(d);
    if (fw > 0) {
        HIP_OK(launch_fill2(w.list, B, -1, w.ctl, kCtlWords, 0, s));
        BpArgs a = bp_args(d, w, syndromes, B);
        a.corr = corrections;
        a.llr_lsd = w.llr;
        a.info = info;
        FuseArgs f;
        memset(&f, 0, sizeof(f));
        f.lsd = lsd_args(d, w, syndromes, w.llr, corrections, info);
        f.lsd.list = w.list;
        f.lsd.list_count = w.ctl + kCtlList;
        f.lsd.bp_iters = d->params.max_iter;
        f.lsd.coherent_llr = 1;
        with_overflow_list(d, w, f.lsd);
        f.list_w = w.list;
        f.tail = w.ctl + kCtlList;
        f.bp_done = w.ctl + kCtlBpDone;
        f.lsd_done = w.ctl + kCtlLsdDone;
        f.lsd_waves = fw;
        f.lsd_bytes = (int)bp_lds_bytes(d->code->g, d->bp_slots, d->bp_se);
        if (timing) HIP_OK(hipEventRecord(d->ev[0], s));
        HIP_OK(launch_bp_fused(a, f, d->lsd_W, bp_grid(d, B), s));
        if (timing) HIP_OK(hipEventRecord(d->ev[1], s));
        // every published entry not marked done (normally none), on a fresh work counter
        LsdArgs rest = f.lsd;
        rest.next_item = w.ctl + kCtlItem2;
        rest.skip_done = 1;
        rest.done_count = w.ctl + kCtlLsdDone;
        rest.coherent_llr = 0;  // after the kernel boundary plain loads see every row
        with_overflow_list(d, w, rest);
        HIP_OK(launch_lsd(rest, d->lsd_W, std::min(d->lsd_grid, d->num_cus), s));
        HIP_OK(run_overflow(d, w, syndromes, w.llr, corrections, info, d->params.max_iter, s));
        if (timing) HIP_OK(hipEventRecord(d->ev[2], s));
        return QLSD_OK;
    }
    HIP_OK(launch_zero(w.ctl, kCtlWords, s));
    BpArgs a = bp_args(d, w, syndromes, B);
    if (timing) HIP_OK(hipEventRecord(d->ev[0], s));
    a.corr = corrections;
    a.llr_lsd = w.llr;
    a.lsd_flag = w.flag;
    a.info = info;
    HIP_OK(run_bp(d, a, B, s));
    if (timing) HIP_OK(hipEventRecord(d->ev[1], s));
    HIP_OK(launch_compact(w.flag, B, w.list, w.ctl + kCtlList, s));
    if (d->net) HIP_OK(net_refine_listed(d->net, d->d_lam, syndromes, w.llr, w.list, w.ctl + kCtlList, B, d->d_netws, s));
    if (d->params.flags & QLSD_FLAG_OSD0_POST) {
        HIP_OK(run_osd0(d, w, syndromes, w.llr, 0, w.list, w.ctl + kCtlList, corrections, info, d->params.max_iter, s,
                        d->params.osd_method == 1 ? d->params.osd_order : 0));
        if (timing) HIP_OK(hipEventRecord(d->ev[2], s));
        return QLSD_OK;
    }
    LsdArgs l = lsd_args(d, w, syndromes, w.llr, corrections, info);
    l.list = w.list;
    l.list_count = w.ctl + kCtlList;
    l.bp_iters = d->params.max_iter;
    with_overflow_list(d, w, l);
    HIP_OK(launch_lsd(l, d->lsd_W, d->lsd_grid, s));
    HIP_OK(run_overflow(d, w, syndromes, w.llr, corrections, info, d->params.max_iter, s));
    if (timing) HIP_OK(hipEventRecord(d->ev[2], s));
    return QLSD_OK;
}

qlsd_status qlsd_decode(qlsd_decoder d, const uint8_t *syndromes, int32_t B, uint8_t *corrections,
                        qlsd_shot_info *info, void *stream) {
    qlsd_status st = check_call(d, syndromes, B, corrections);
    if (st != QLSD_OK || B == 0) return st;
    return decode_with(d, decoder_ws(d), syndromes, B, corrections, info, (hipStream_t)stream,
                       d->timing && d->timing_on);
}

// Device address of this device's `scratch` (looked up once per device, with it current).
static qlsd_status static_scratch(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kStaticMaxDevices) return fail(QLSD_E_DEVICE, "device %d beyond the static scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(QLSD_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = (unsigned char *)p;
    }
    *out = g_scratch_dev[dev];
    return QLSD_OK;
}

qlsd_status qlsd_decode_static(qlsd_decoder d, const uint8_t *syndromes, int32_t B, uint8_t *corrections,
                               qlsd_shot_info *info, void *stream) {
    qlsd_status st = check_call(d, syndromes, B, corrections);
    if (st != QLSD_OK || B == 0) return st;
    if (d->netws_bytes) return fail(QLSD_E_UNSUPPORTED, "qlsd_decode_static: the attached net needs a device workspace");
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev != d->code->device) return fail(QLSD_E_INVALID, "decoder lives on device %d, current is %d", d->code->device, dev);
    const size_t n = (size_t)d->code->g.n;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t o_ctl = take(sizeof(int) * kCtlWords), o_flag = take((size_t)B), o_list = take(sizeof(int) * (size_t)B),
                 o_llr = take(sizeof(float) * (size_t)B * n);
    const bool two = d->mid && d->wide;
    const bool wws = d->wide || ((d->params.flags & QLSD_FLAG_OSD0_POST) && d->osd_W == kWideW);
    const size_t o_ovf = d->ovf ? take(sizeof(int) * (size_t)B) : 0;
    const size_t o_ovf2 = two ? take(sizeof(int) * (size_t)B) : 0;
    const size_t o_wide = wws ? take(sizeof(uint64_t) * lsd_wide_ws_words() * kStaticWideGrid) : 0;
    if (off > kStaticScratchBytes)
        return fail(QLSD_E_BATCH, "qlsd_decode_static: B=%d needs %zu bytes of scratch, the library holds %zu",
                    B, off, kStaticScratchBytes);
    unsigned char *base = nullptr;
    st = static_scratch(dev, &base);
    if (st != QLSD_OK) return st;
    Ws w;
    w.ctl = (int *)(base + o_ctl);
    w.flag = base + o_flag;
    w.list = (int *)(base + o_list);
    w.llr = (float *)(base + o_llr);
    w.ovf_list = d->ovf ? (int *)(base + o_ovf) : nullptr;
    w.ovf2_list = two ? (int *)(base + o_ovf2) : nullptr;
    w.wide_ws = wws ? (uint64_t *)(base + o_wide) : nullptr;
    w.wide_grid = kStaticWideGrid;
    return decode_with(d, w, syndromes, B, corrections, info, (hipStream_t)stream, false);
}

qlsd_status qlsd_bp(qlsd_decoder d, const uint8_t *syndromes, int32_t B, float *llr_out, uint8_t *hard_out,
                    qlsd_shot_info *info, void *stream) {
    qlsd_status st = check_call(d, syndromes, B, llr_out);
    if (st != QLSD_OK || B == 0) return st;
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(launch_zero(d->d_ctl, kCtlWords, s));
    BpArgs a = bp_args(d, decoder_ws(d), syndromes, B);
    a.corr = hard_out;
    a.llr_out = llr_out;
    a.info = info;
    HIP_OK(run_bp(d, a, B, s));
    return QLSD_OK;
}

qlsd_status qlsd_lsd(qlsd_decoder d, const uint8_t *syndromes, const float *llr, int32_t B,
                     uint8_t *corrections, qlsd_shot_info *info, void *stream) {
    qlsd_status st = check_call(d, syndromes, B, corrections);
    if (st != QLSD_OK || B == 0) return st;
    if (!llr) return fail(QLSD_E_INVALID, "llr is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(launch_zero(d->d_ctl, kCtlWords, s));
    const Ws w = decoder_ws(d);
    LsdArgs l = lsd_args(d, w, syndromes, llr, corrections, info);
    l.count = B;
    with_overflow_list(d, w, l);
    HIP_OK(launch_lsd(l, d->lsd_W, std::min(d->lsd_grid, (B + 3) / 4), s));
    HIP_OK(run_overflow(d, w, syndromes, llr, corrections, info, 0, s));
    return QLSD_OK;
}

qlsd_status qlsd_lsd_stats(qlsd_decoder d, const uint8_t *syndromes, const float *llr, int32_t B,
                           uint8_t *corrections, qlsd_shot_info *info, qlsd_cluster_stats *stats, void *stream) {
    qlsd_status st = check_call(d, syndromes, B, corrections);
    if (st != QLSD_OK || B == 0) return st;
    if (!llr || !stats) return fail(QLSD_E_INVALID, "llr or stats is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(launch_zero(d->d_ctl, kCtlWords, s));
    const Ws w = decoder_ws(d);
    LsdArgs l = lsd_args(d, w, syndromes, llr, corrections, info);
    l.count = B;
    l.cstats = stats;
    with_overflow_list(d, w, l);
    HIP_OK(launch_lsd(l, d->lsd_W, std::min(d->lsd_grid, (B + 3) / 4), s));
    HIP_OK(run_overflow(d, w, syndromes, llr, corrections, info, 0, s, stats));
    return QLSD_OK;
}

qlsd_status qlsd_error_clusters(qlsd_code code, const uint8_t *errors, int32_t B, qlsd_cluster_stats *stats,
                                void *stream) {
    g_err[0] = 0;
    if (!code || B < 0 || (B > 0 && (!errors || !stats))) return fail(QLSD_E_INVALID, "bad error-cluster call");
    if (B == 0) return QLSD_OK;
    if (sizeof(int32_t) * (2 * (size_t)code->g.n + code->g.m) > kLdsPerCu - 1024)
        return fail(QLSD_E_UNSUPPORTED, "graph too large for the error-cluster kernel");
    HIP_OK(launch_error_clusters(code->g, errors, B, stats, (hipStream_t)stream));
    return QLSD_OK;
}

qlsd_status qlsd_osd0(qlsd_decoder d, const uint8_t *syndromes, const float *llr, int32_t B,
                      uint8_t *corrections, qlsd_shot_info *info, void *stream) {
    qlsd_status st = check_call(d, syndromes, B, corrections);
    if (st != QLSD_OK || B == 0) return st;
    if (!llr) return fail(QLSD_E_INVALID, "llr is NULL");
    if (!d->osd_ok)
        return fail(QLSD_E_UNSUPPORTED, "OSD-0 supports n <= %d and m <= %d (n=%d, m=%d)", kOsdMaxSort, kWideRows,
                    d->code->g.n, d->code->g.m);
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(launch_zero(d->d_ctl, kCtlWords, s));
    HIP_OK(run_osd0(d, decoder_ws(d), syndromes, llr, B, nullptr, nullptr, corrections, info, 0, s));
    return QLSD_OK;
}

qlsd_status qlsd_osd_cs(qlsd_decoder d, const uint8_t *syndromes, const float *llr, int32_t B, int32_t order,
                        uint8_t *corrections, qlsd_shot_info *info, void *stream) {
    qlsd_status st = check_call(d, syndromes, B, corrections);
    if (st != QLSD_OK) return st;
    if (order < 1 || order > kOsdCsMaxOrder) return fail(QLSD_E_INVALID, "OSD-CS order must be in [1, %d]", kOsdCsMaxOrder);
    if (B == 0) return QLSD_OK;
    if (!llr) return fail(QLSD_E_INVALID, "llr is NULL");
    if (!d->osd_cs_ok)
        return fail(QLSD_E_UNSUPPORTED, "global OSD-CS supports n <= %d and m <= 256 (n=%d, m=%d)", kOsdMaxSort,
                    d->code->g.n, d->code->g.m);
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(launch_zero(d->d_ctl, kCtlWords, s));
    HIP_OK(run_osd0(d, decoder_ws(d), syndromes, llr, B, nullptr, nullptr, corrections, info, 0, s, order));
    return QLSD_OK;
}

// Sets the LSD kernel's local-row capacity to 64 * W (W in {1, 2, 4}); shots that outgrow it go
// to the overflow kernels, whose buffers are allocated here when first needed.  Returns false (and
// leaves the decoder as it was) when W does not fit the LDS budget, no overflow kernel fits the
// code, or an allocation fails.
static bool set_lsd_capacity(qlsd_decoder d, int W) {
    const DevGraph &g = d->code->g;
    const bool with_mu = d->params.lsd_order > 0;
    if (with_mu && W != 4) return false;  // LSD-mu kernels are built for W = 4 only
    if (lsd_total_lds(g, W, d->lsd_keys_in_lds != 0, d->lsd_graph_in_lds != 0, with_mu) > kLdsPerCu - 1024) return false;
    if (!configure_overflow(d, W, true)) return false;
    d->lsd_W = W;
    d->lsd_wave_bytes = (int)lsd_wave_bytes(g, W, d->lsd_keys_in_lds != 0, with_mu);
    return true;
}

qlsd_status qlsd_decoder_set_lsd_capacity(qlsd_decoder d, int32_t local_rows) {
    if (!d) return fail(QLSD_E_INVALID, "null decoder");
    if (local_rows != 64 && local_rows != 128 && local_rows != 256)
        return fail(QLSD_E_INVALID, "LSD capacity must be 64, 128 or 256 local rows (got %d)", local_rows);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != d->code->device)
        return fail(QLSD_E_INVALID, "decoder lives on device %d, current is %d", d->code->device, dev);
    if (!set_lsd_capacity(d, local_rows / 64))
        return fail(QLSD_E_UNSUPPORTED, "LSD capacity %d: %s", local_rows,
                    d->params.lsd_order > 0 ? "LSD-mu decoders run with 256 local rows"
                                            : "no overflow kernel fits this code, or an allocation failed");
    return QLSD_OK;
}

qlsd_status qlsd_decoder_set_lsd_schedule(qlsd_decoder d, int32_t schedule) {
    if (!d) return fail(QLSD_E_INVALID, "null decoder");
    if (schedule != QLSD_LSD_PER_COLUMN && schedule != QLSD_LSD_CLUSTER_BATCHED)
        return fail(QLSD_E_INVALID, "unknown LSD schedule %d", schedule);
    if (schedule == QLSD_LSD_CLUSTER_BATCHED && d->lsd_W != 4)
        return fail(QLSD_E_UNSUPPORTED, "the cluster-batched schedule runs in the 256-row LSD kernel (capacity is %d)",
                    64 * d->lsd_W);
    d->lsd_cb = schedule == QLSD_LSD_CLUSTER_BATCHED;
    return QLSD_OK;
}

qlsd_status qlsd_decoder_tune(qlsd_decoder d, const uint8_t *syndromes, int32_t B, int32_t reps, void *stream,
                              char *report, int32_t report_len) {
    qlsd_status st = check_call(d, syndromes, B, syndromes);
    if (st != QLSD_OK) return st;
    if (B == 0 || reps < 1) return fail(QLSD_E_INVALID, "need B >= 1 and reps >= 1");
    hipStream_t s = (hipStream_t)stream;
    const DevGraph &g = d->code->g;
    std::string rep;
    char line[160];
    uint8_t *corr = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        hipFree(corr);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
    };
    if (hipMalloc((void **)&corr, (size_t)B * g.n) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(QLSD_E_NOMEM, "tuning scratch allocation failed");
    }
    // average device time (ms) of `reps` runs of f after one warm-up run
    auto timeit = [&](auto &&f) -> float {
        if (f() != hipSuccess) return -1.f;
        hipEventRecord(e0, s);
        for (int r = 0; r < reps; r++)
            if (f() != hipSuccess) return -1.f;
        hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) return -1.f;
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        return ms / reps;
    };
    auto bp_run = [&]() -> hipError_t {
        hipError_t e = launch_zero(d->d_ctl, kCtlWords, s);
        if (e != hipSuccess) return e;
        BpArgs a = bp_args(d, decoder_ws(d), syndromes, B);
        a.corr = corr;
        a.llr_lsd = d->d_llr;
        a.lsd_flag = d->d_flag;
        return run_bp(d, a, B, s);
    };
    // Whole decode (qlsd_decode: BP and LSD in one kernel where the shape allows it, else the
    // separate kernels), the measure of a BP shape when no refinement net is attached: the
    // one-kernel path needs at most 4 workgroups per CU, so BP alone would favour shapes that
    // lose it.
    auto decode_run = [&]() -> hipError_t {
        return qlsd_decode(d, syndromes, B, corr, nullptr, stream) == QLSD_OK ? hipSuccess : hipErrorUnknown;
    };
    // BP with shot slots: the largest slot count that fits each workgroups-per-CU tier
    if (!d->bp_graph) {
        int best_S = d->bp_slots, best_grid = d->bp_grid, best_se = d->bp_se;
        float best = 1e30f;
        for (int wg : {1, 2, 3, 4, 5, 6, 8}) {
            const size_t budget = kLdsPerCu / wg - 512;
            int S = kMaxSlots;
            while (S > 0 && bp_lds_bytes(g, S, bp_min_stride(g)) > budget) S--;
            if (S < 4) continue;
            d->bp_slots = S;
            d->bp_grid = wg * d->num_cus;
            d->bp_se = bp_stride_for(d->code, S, budget);
            const bool whole = d->net == nullptr;
            const float ms = whole ? timeit(decode_run) : timeit(bp_run);
            snprintf(line, sizeof(line), "%s slots %d x %d workgroups/CU: %.4f ms\n",
                     whole ? (fuse_waves(d) > 0 ? "decode (BP + LSD one kernel)," : "decode (BP, LSD),") : "bp",
                     S, wg, ms);
            rep += line;
            if (ms > 0.f && ms < best) { best = ms; best_S = S; best_grid = d->bp_grid; best_se = d->bp_se; }
        }
        d->bp_slots = best_S;
        d->bp_grid = best_grid;
        d->bp_se = best_se;
        snprintf(line, sizeof(line), "bp chosen: slots %d, grid %d\n", best_S, best_grid);
        rep += line;
    }
    // LSD on the shots this BP leaves unsolved
    if (bp_run() != hipSuccess || launch_compact(d->d_flag, B, d->d_list, d->d_ctl + kCtlList, s) != hipSuccess) {
        cleanup();
        return fail(QLSD_E_DEVICE, "tuning launch failed");
    }
    int best_lsd = d->lsd_grid;
    float best = 1e30f;
    for (int mult : {2, 4, 8, 16, 32}) {
        const int grid = mult * d->num_cus;
        auto lsd_run = [&]() -> hipError_t {
            hipError_t e = launch_zero(d->d_ctl + kCtlItem, 1, s);
            if (e != hipSuccess) return e;
            LsdArgs l = lsd_args(d, decoder_ws(d), syndromes, d->d_llr, corr, nullptr);
            l.list = d->d_list;
            l.list_count = d->d_ctl + kCtlList;
            l.bp_iters = d->params.max_iter;
            return launch_lsd(l, d->lsd_W, grid, s);
        };
        const float ms = timeit(lsd_run);
        snprintf(line, sizeof(line), "lsd %d workgroups: %.4f ms\n", grid, ms);
        rep += line;
        if (ms > 0.f && ms < best) { best = ms; best_lsd = grid; }
    }
    d->lsd_grid = best_lsd;
    snprintf(line, sizeof(line), "lsd chosen: %d workgroups\n", best_lsd);
    rep += line;
    // LSD capacity per wavefront (the schedule for uneven cluster sizes): every tier up to the
    // default, shots beyond a smaller tier's capacity decoded again by the overflow kernels; timed
    // on the whole decode (the tier also decides whether BP and LSD share a kernel)
    {
        const int W0 = d->lsd_W;
        int best_W = W0;
        // A tier below the default re-decodes the shots that outgrow it after the LSD kernel; one
        // sample batch may hold fewer of them than other batches will, so such a tier must beat
        // the default by kCapacityMargin to be kept
        constexpr float kCapacityMargin = 0.9f;
        float ms_w[3] = {0.f, 0.f, 0.f};
        for (int k = 2; k >= 0; k--) {
            const int W = 1 << k;
            if (W > W0 || !set_lsd_capacity(d, W)) continue;
            ms_w[k] = timeit(decode_run);
            snprintf(line, sizeof(line), "lsd capacity %d local rows per wavefront: decode %.4f ms\n", 64 * W, ms_w[k]);
            rep += line;
        }
        const int k0 = W0 == 4 ? 2 : W0 == 2 ? 1 : 0;
        float best_ms = ms_w[k0] > 0.f ? ms_w[k0] : 1e30f;
        for (int k = 0; k < k0; k++)
            if (ms_w[k] > 0.f && ms_w[k] < kCapacityMargin * ms_w[k0] && ms_w[k] < best_ms) {
                best_ms = ms_w[k];
                best_W = 1 << k;
            }
        set_lsd_capacity(d, best_W);
        snprintf(line, sizeof(line), "lsd capacity chosen: %d local rows\n", 64 * best_W);
        rep += line;
    }
    // LSD schedule of the 256-row kernel: columns one at a time, or batched across the clusters
    // that grow in the same round (kept only when 2 % faster: it costs registers)
    if (d->lsd_W == 4) {
        d->lsd_cb = false;
        const float ms0 = timeit(decode_run);
        d->lsd_cb = true;
        const float ms1 = timeit(decode_run);
        d->lsd_cb = ms1 > 0.f && ms0 > 0.f && ms1 < 0.98f * ms0;
        snprintf(line, sizeof(line), "lsd schedule per column: decode %.4f ms; batched across clusters: %.4f ms\n", ms0, ms1);
        rep += line;
        snprintf(line, sizeof(line), "lsd schedule chosen: %s\n", d->lsd_cb ? "batched across clusters" : "per column");
        rep += line;
    }
    const hipError_t e = hipStreamSynchronize(s);
    cleanup();
    if (e != hipSuccess) return fail(QLSD_E_DEVICE, "tuning failed: %s", hipGetErrorString(e));
    if (report && report_len > 0) {
        const size_t k = std::min<size_t>(rep.size(), (size_t)report_len - 1);
        memcpy(report, rep.data(), k);
        report[k] = 0;
    }
    return QLSD_OK;
}

qlsd_status qlsd_decoder_stage_ms(qlsd_decoder d, float *bp_ms, float *lsd_ms) {
    g_err[0] = 0;
    if (!d) return fail(QLSD_E_INVALID, "decoder is NULL");
    if (!d->timing) return fail(QLSD_E_INVALID, "decoder was created without QLSD_FLAG_STAGE_TIMING");
    HIP_OK(hipEventSynchronize(d->ev[2]));
    float a = 0.f, b = 0.f;
    HIP_OK(hipEventElapsedTime(&a, d->ev[0], d->ev[1]));
    HIP_OK(hipEventElapsedTime(&b, d->ev[1], d->ev[2]));
    if (bp_ms) *bp_ms = a;
    if (lsd_ms) *lsd_ms = b;
    return QLSD_OK;
}

qlsd_status qlsd_decoder_set_stage_timing(qlsd_decoder d, int32_t enable) {
    g_err[0] = 0;
    if (!d) return fail(QLSD_E_INVALID, "decoder is NULL");
    if (!d->timing) return fail(QLSD_E_INVALID, "decoder was created without QLSD_FLAG_STAGE_TIMING");
    d->timing_on = enable != 0;
    return QLSD_OK;
}

qlsd_status qlsd_decoder_set_net(qlsd_decoder d, qlsd_net net) {
    g_err[0] = 0;
    if (!d) return fail(QLSD_E_INVALID, "decoder is NULL");
    if (net) {
        int m = 0, n = 0;
        net_graph_dims(net, &m, &n);
        if (m != d->code->g.m || n != d->code->g.n)
            return fail(QLSD_E_INVALID, "net built for a %dx%d code, the decoder's is %dx%d", m, n, d->code->g.m, d->code->g.n);
    }
    // large graphs: the decoder gets its own feature workspace, so decoders sharing one net may
    // run concurrently on different streams
    const size_t need = net ? net_infer_workspace_bytes(net) : 0;
    if (need != d->netws_bytes) {
        if (d->d_netws) {
            hipDeviceSynchronize();
            hipFree(d->d_netws);
        }
        d->d_netws = nullptr;
        d->netws_bytes = 0;
        if (need) {
            if (hipMalloc((void **)&d->d_netws, need) != hipSuccess) {
                d->d_netws = nullptr;
                d->net = nullptr;
                return fail(QLSD_E_NOMEM, "device allocation of the refinement workspace failed");
            }
            d->netws_bytes = need;
        }
    }
    d->net = net;
    return QLSD_OK;
}

qlsd_status qlsd_sync(qlsd_decoder d) {
    g_err[0] = 0;
    if (!d) return fail(QLSD_E_INVALID, "decoder is NULL");
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipGetLastError());
    return QLSD_OK;
}

}  // extern "C"
