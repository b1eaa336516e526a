// Overlapping-window decoding (include/qlsd_window.h): host-side window construction, then per
// window three small kernels around an ordinary qlsd_decode -- gather the window's syndrome rows
// from the running residual, decode, commit the window's first c rounds of faults and refresh
// the residual of every detector those faults touch.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/qlsd_window.h"
#include "qlsd_internal.h"

using namespace qlsd;

namespace {

struct Window {
    qlsd_code code = nullptr;
    qlsd_decoder dec = nullptr;
    int rows = 0, cols = 0, n_commit = 0, n_touch = 0;
    int32_t *d_rows = nullptr;    // rows: full-H detector of each window row
    int32_t *d_commit = nullptr;  // n_commit pairs (window column, full-H fault) committed here
    int32_t *d_touch = nullptr;   // n_touch: detectors whose residual the committed faults change
};

// s_w[b][r] = res[b][rows[r]]
__global__ void gather_kernel(const uint8_t *res, int m, const int32_t *rows, int nr, int B, uint8_t *s_w) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * nr) return;
    const int64_t b = t / nr;
    s_w[t] = res[b * m + rows[t % nr]];
}

// corr[b][fault] = e_w[b][window column] for the committed pairs
__global__ void commit_kernel(const uint8_t *e_w, int nc, const int32_t *pairs, int np, int n, int B, uint8_t *corr) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * np) return;
    const int64_t b = t / np;
    const int q = (int)(t % np);
    corr[b * n + pairs[2 * q + 1]] = e_w[b * nc + pairs[2 * q]];
}

// res[b][i] = s[b][i] xor (H corr[b])_i for the listed detectors
__global__ void refresh_kernel(const uint8_t *s, const uint8_t *corr, const int32_t *row_ptr, const int32_t *col_idx,
                               int m, int n, const int32_t *touch, int nt, int B, uint8_t *res) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * nt) return;
    const int64_t b = t / nt;
    const int i = touch[t % nt];
    uint8_t acc = s[b * m + i];
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; e++) acc ^= corr[b * n + col_idx[e]];
    res[b * m + i] = acc & 1;
}

__global__ void copy_kernel(const uint8_t *a, uint8_t *b, int64_t count) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) b[t] = a[t];
}

__global__ void zero_kernel(uint8_t *a, int64_t count) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) a[t] = 0;
}

inline unsigned blocks(int64_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

struct qlsd_window_s {
    qlsd_code code;
    DevGraph g;
    int max_batch;
    std::vector<Window> win;
    uint8_t *d_res = nullptr;   // max_batch x m: running residual syndrome
    uint8_t *d_sw = nullptr;    // max_batch x max rows
    uint8_t *d_ew = nullptr;    // max_batch x max cols
};

extern "C" {

qlsd_status qlsd_window_create(qlsd_code code, const double *priors, const int32_t *det_round, int32_t w,
                               int32_t c, const qlsd_params *params, int32_t max_batch, qlsd_window *out) {
    set_last_error("");
    if (!out) return QLSD_E_INVALID;
    *out = nullptr;
    if (!code || !priors || !det_round || !params || c < 1 || w <= c || max_batch < 1) {
        set_last_error("window: bad arguments (need 1 <= c < w, max_batch >= 1)");
        return QLSD_E_INVALID;
    }
    const DevGraph g = code_graph(code);
    const int m = g.m, n = g.n;
    std::vector<int32_t> rp(m + 1), ci(g.nnz);
    if (hipMemcpy(rp.data(), g.row_ptr, sizeof(int32_t) * (m + 1), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(ci.data(), g.col_idx, sizeof(int32_t) * g.nnz, hipMemcpyDeviceToHost) != hipSuccess) {
        set_last_error("window: reading H back failed");
        return QLSD_E_DEVICE;
    }
    int n_rounds = 0;
    for (int i = 0; i < m; i++) {
        if (det_round[i] < 0) { set_last_error("window: negative detector round"); return QLSD_E_INVALID; }
        n_rounds = std::max(n_rounds, det_round[i] + 1);
    }
    std::vector<int> fr(n, 1 << 30);
    for (int i = 0; i < m; i++)
        for (int e = rp[i]; e < rp[i + 1]; e++) fr[ci[e]] = std::min(fr[ci[e]], det_round[i]);
    // the scheme's windows: [k, k + w) every c rounds while another fits, then [k, n_rounds)
    std::vector<int> lo, hi, cm;
    for (int k = 0;; k += c) {
        if (k + w < n_rounds) { lo.push_back(k); hi.push_back(k + w); cm.push_back(k + c); continue; }
        lo.push_back(k); hi.push_back(n_rounds); cm.push_back(n_rounds);
        break;
    }
    qlsd_window wd = new (std::nothrow) qlsd_window_s();
    if (!wd) return QLSD_E_NOMEM;
    wd->code = code;
    wd->g = g;
    wd->max_batch = max_batch;
    int max_rows = 1, max_cols = 1;
    qlsd_status st = QLSD_OK;
    std::vector<int> col_pos(n);
    for (size_t k = 0; k < lo.size() && st == QLSD_OK; k++) {
        std::vector<int32_t> rows, cols;
        for (int i = 0; i < m; i++)
            if (det_round[i] >= lo[k] && det_round[i] < hi[k]) rows.push_back(i);
        for (int j = 0; j < n; j++)
            if (fr[j] >= lo[k] && fr[j] < hi[k]) { col_pos[j] = (int)cols.size(); cols.push_back(j); }
            else col_pos[j] = -1;
        // window sub-matrix, CSR over its rows
        std::vector<int32_t> wrp(1, 0), wci;
        for (int i : rows) {
            for (int e = rp[i]; e < rp[i + 1]; e++)
                if (col_pos[ci[e]] >= 0) wci.push_back(col_pos[ci[e]]);
            wrp.push_back((int32_t)wci.size());
        }
        std::vector<double> wp(cols.size());
        for (size_t q = 0; q < cols.size(); q++) wp[q] = priors[cols[q]];
        std::vector<int32_t> pairs, touch;
        std::vector<char> touched(m, 0);
        for (size_t q = 0; q < cols.size(); q++)
            if (fr[cols[q]] < cm[k]) {
                pairs.push_back((int32_t)q);
                pairs.push_back(cols[q]);
            }
        // detectors whose residual the committed faults can change (CSC walk via the CSR)
        std::vector<char> committed(n, 0);
        for (size_t q = 0; q + 1 < pairs.size(); q += 2) committed[pairs[q + 1]] = 1;
        for (int i = 0; i < m; i++)
            for (int e = rp[i]; e < rp[i + 1]; e++)
                if (committed[ci[e]]) { touched[i] = 1; break; }
        for (int i = 0; i < m; i++)
            if (touched[i]) touch.push_back(i);
        Window W;
        W.rows = (int)rows.size();
        W.cols = (int)cols.size();
        W.n_commit = (int)pairs.size() / 2;
        W.n_touch = (int)touch.size();
        st = qlsd_code_create(W.rows, W.cols, (int64_t)wci.size(), wrp.data(), wci.data(), &W.code);
        if (st == QLSD_OK) st = qlsd_decoder_create(W.code, params, wp.data(), max_batch, &W.dec);
        if (st == QLSD_OK) {
            hipError_t e = hipMalloc((void **)&W.d_rows, sizeof(int32_t) * std::max<size_t>(1, rows.size()));
            if (e == hipSuccess) e = hipMalloc((void **)&W.d_commit, sizeof(int32_t) * std::max<size_t>(2, pairs.size()));
            if (e == hipSuccess) e = hipMalloc((void **)&W.d_touch, sizeof(int32_t) * std::max<size_t>(1, touch.size()));
            if (e == hipSuccess && !rows.empty())
                e = hipMemcpy(W.d_rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice);
            if (e == hipSuccess && !pairs.empty())
                e = hipMemcpy(W.d_commit, pairs.data(), sizeof(int32_t) * pairs.size(), hipMemcpyHostToDevice);
            if (e == hipSuccess && !touch.empty())
                e = hipMemcpy(W.d_touch, touch.data(), sizeof(int32_t) * touch.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) { set_last_error("window: device allocation failed"); st = QLSD_E_NOMEM; }
        }
        max_rows = std::max(max_rows, W.rows);
        max_cols = std::max(max_cols, W.cols);
        wd->win.push_back(W);
    }
    if (st == QLSD_OK) {
        hipError_t e = hipMalloc((void **)&wd->d_res, (size_t)max_batch * m);
        if (e == hipSuccess) e = hipMalloc((void **)&wd->d_sw, (size_t)max_batch * max_rows);
        if (e == hipSuccess) e = hipMalloc((void **)&wd->d_ew, (size_t)max_batch * max_cols);
        if (e != hipSuccess) { set_last_error("window: device allocation failed"); st = QLSD_E_NOMEM; }
    }
    if (st != QLSD_OK) {
        char msg[512];
        strncpy(msg, qlsd_last_error(), sizeof(msg) - 1);
        msg[sizeof(msg) - 1] = 0;
        qlsd_window_destroy(wd);
        set_last_error("%s", msg);
        return st;
    }
    *out = wd;
    return QLSD_OK;
}

qlsd_status qlsd_window_decode(qlsd_window wd, const uint8_t *syndromes, int32_t B, uint8_t *corrections,
                               void *stream) {
    set_last_error("");
    if (!wd) return QLSD_E_INVALID;
    if (B < 0 || B > wd->max_batch) { set_last_error("window: B outside [0, max_batch]"); return QLSD_E_BATCH; }
    if (B == 0) return QLSD_OK;
    if (!syndromes || !corrections) { set_last_error("window: NULL syndromes or corrections"); return QLSD_E_INVALID; }
    hipStream_t s = (hipStream_t)stream;
    const int m = wd->g.m, n = wd->g.n;
    hipLaunchKernelGGL(copy_kernel, dim3(blocks((int64_t)B * m)), dim3(256), 0, s, syndromes, wd->d_res, (int64_t)B * m);
    hipLaunchKernelGGL(zero_kernel, dim3(blocks((int64_t)B * n)), dim3(256), 0, s, corrections, (int64_t)B * n);
    for (const Window &W : wd->win) {
        hipLaunchKernelGGL(gather_kernel, dim3(blocks((int64_t)B * W.rows)), dim3(256), 0, s, wd->d_res, m, W.d_rows,
                           W.rows, B, wd->d_sw);
        qlsd_status st = qlsd_decode(W.dec, wd->d_sw, B, wd->d_ew, nullptr, stream);
        if (st != QLSD_OK) return st;
        if (W.n_commit)
            hipLaunchKernelGGL(commit_kernel, dim3(blocks((int64_t)B * W.n_commit)), dim3(256), 0, s, wd->d_ew, W.cols,
                               W.d_commit, W.n_commit, n, B, corrections);
        if (W.n_touch)
            hipLaunchKernelGGL(refresh_kernel, dim3(blocks((int64_t)B * W.n_touch)), dim3(256), 0, s, syndromes,
                               corrections, wd->g.row_ptr, wd->g.col_idx, m, n, W.d_touch, W.n_touch, B, wd->d_res);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_last_error("window: %s", hipGetErrorString(e)); return QLSD_E_DEVICE; }
    return QLSD_OK;
}

int32_t qlsd_window_count(qlsd_window wd) { return wd ? (int32_t)wd->win.size() : 0; }

void qlsd_window_destroy(qlsd_window wd) {
    if (!wd) return;
    for (Window &W : wd->win) {
        qlsd_decoder_destroy(W.dec);
        qlsd_code_destroy(W.code);
        hipFree(W.d_rows);
        hipFree(W.d_commit);
        hipFree(W.d_touch);
    }
    hipFree(wd->d_res);
    hipFree(wd->d_sw);
    hipFree(wd->d_ew);
    delete wd;
}

}  // extern "C"
