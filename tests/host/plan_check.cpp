// Host-side check of the BP kernels' launch planning (no GPU needed): reads a CSR graph, runs the
// library's large-graph message layout builder and the slot kernel's message stride chooser, and
// prints what the test asserts on.
//   plan_check layout <graph>              -> "words W consistent C fault F check K"
//   plan_check stride <graph> <S> <budget> -> "stride SE bytes B"
// Graph file: "m n nnz", then nnz column indices (CSR order), then m + 1 row pointers.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <set>
#include <vector>

#include "qlsd_internal.h"

int main(int argc, char **argv) {
    if (argc < 3) return 1;
    FILE *f = fopen(argv[2], "r");
    if (!f) return 1;
    int m, n, E;
    if (fscanf(f, "%d %d %d", &m, &n, &E) != 3) return 1;
    std::vector<int> ci(E), rp(m + 1);
    for (int e = 0; e < E; e++)
        if (fscanf(f, "%d", &ci[e]) != 1) return 1;
    for (int i = 0; i <= m; i++)
        if (fscanf(f, "%d", &rp[i]) != 1) return 1;
    fclose(f);
    std::vector<int> cp(n + 1, 0), fill(n, 0), row_edge(E), col_edge(E);
    for (int e = 0; e < E; e++) cp[ci[e] + 1]++;
    for (int j = 0; j < n; j++) cp[j + 1] += cp[j];
    for (int i = 0; i < m; i++)
        for (int e = rp[i]; e < rp[i + 1]; e++) {
            const int k = cp[ci[e]] + fill[ci[e]]++;
            col_edge[k] = e;
            row_edge[e] = k;
        }
    qlsd::DevGraph g;
    memset(&g, 0, sizeof(g));
    g.m = m;
    g.n = n;
    g.nnz = E;
    g.max_rw = g.max_cw = 0;
    g.min_rw = g.min_cw = 1 << 30;
    for (int i = 0; i < m; i++) g.max_rw = std::max(g.max_rw, rp[i + 1] - rp[i]), g.min_rw = std::min(g.min_rw, rp[i + 1] - rp[i]);
    for (int j = 0; j < n; j++) g.max_cw = std::max(g.max_cw, cp[j + 1] - cp[j]), g.min_cw = std::min(g.min_cw, cp[j + 1] - cp[j]);
    if (!strcmp(argv[1], "stride")) {
        if (argc < 5) return 1;
        const int S = atoi(argv[3]);
        const size_t budget = (size_t)atol(argv[4]);
        const int se = qlsd::bp_msg_stride(g, rp.data(), cp.data(), col_edge.data(), S, budget);
        printf("stride %d bytes %zu\n", se, qlsd::bp_lds_bytes(g, S, se));
        return 0;
    }
    // the library's orders: decreasing weight, ties by index
    auto order = [](const std::vector<int> &ptr, int cnt) {
        std::vector<int> o(cnt);
        for (int x = 0; x < cnt; x++) o[x] = x;
        std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return ptr[a + 1] - ptr[a] > ptr[b + 1] - ptr[b]; });
        return o;
    };
    const std::vector<int> fo = order(cp, n), co = order(rp, m);
    std::vector<int32_t> fm;
    std::vector<uint16_t> rm;
    const int W = qlsd::bp_graph2_layout(m, n, E, rp.data(), cp.data(), row_edge.data(), fo.data(), co.data(), fm, rm);
    if (W <= 0) {
        printf("words %d consistent 0 fault 0 check 0\n", W);
        return 0;
    }
    // every fault entry at a distinct word below W; every check visits exactly its own edges' words
    bool ok = true;
    std::vector<int> owner(W, -1);
    for (int j = 0; j < n && ok; j++)
        for (int u = 0; u < cp[j + 1] - cp[j]; u++) {
            const int w = fm[j] + 64 * u;
            if (w < 0 || w >= W || owner[w] >= 0) { ok = false; break; }
            owner[w] = cp[j] + u;
        }
    for (int i = 0; i < m && ok; i++) {
        std::multiset<int> a, b;
        for (int e = rp[i]; e < rp[i + 1]; e++) {
            a.insert(fm[ci[e]] + 64 * (row_edge[e] - cp[ci[e]]));
            b.insert(rm[e]);
        }
        ok = a == b;
    }
    // modelled LDS cycles per half-wavefront access (32 lanes on 32 four-byte banks)
    long long fc = 0, fa = 0, cc = 0, ca = 0;
    for (int p0 = 0; p0 < n; p0 += 32)
        for (int u = 0; u < g.max_cw; u++) {
            int cnt[32] = {0}, mx = 0;
            for (int p = p0; p < std::min(n, p0 + 32); p++)
                if (u < cp[fo[p] + 1] - cp[fo[p]]) mx = std::max(mx, ++cnt[(fm[fo[p]] + 64 * u) & 31]);
            if (mx) fc += mx, fa++;
        }
    for (int p0 = 0; p0 < m; p0 += 32)
        for (int u = 0; u < g.max_rw; u++) {
            int cnt[32] = {0}, mx = 0;
            for (int p = p0; p < std::min(m, p0 + 32); p++)
                if (u < rp[co[p] + 1] - rp[co[p]]) mx = std::max(mx, ++cnt[rm[rp[co[p]] + u] & 31]);
            if (mx) cc += mx, ca++;
        }
    printf("words %d consistent %d fault %.4f check %.4f\n", W, ok ? 1 : 0, (double)fc / fa, (double)cc / ca);
    return 0;
}
