// Runs the 4-cycle kernels of the library (their source, extracted by the test) on
// host threads over a small graph, with the class bounds and table sizes of the
// library's launches, and compares every vertex's 4-cycle credits with a direct
// sequential count over the same per-slot wedge runs.
// usage: sweep_host graph.bin heavy_k
#include "host_lanes.hpp"
#include <functional>
#include <numeric>
struct int2 { i32 x, y; };
struct int4 { i32 x, y, z, w; };
inline int2 make_int2(i32 a, i32 b) { return int2{a, b}; }
struct GraphStats { int dmax, dplus_max, err, pad, bad_input, pad2; long long pairs; int cnt[16]; long long work[16]; long long slots[16]; };
enum WorkClass { WC_TRI_WAVE = 0, WC_TRI_THREAD, WC_TRI_BLOCK, WC_TRI_LARGE, WC_QL_WAVE, WC_QL_BLOCK, WC_QL_GLOBAL,
                 WC_QH_WAVE, WC_QH_BLOCK, WC_QH_DENSE, WC_QH_GLOBAL, WC_TRI_GROUP, WC_COUNT };
#define QL_WAVE_HC 4096
#define QL_WAVE_DC 64
#define QL_BLOCK_HC 16384
#define QH_WAVE_HC 4096
#define QH_BLOCK_HC 8192
#define QH_PART_ROWS 64
#define QH_DENSE_K 32768
struct DevGraph {
    i32 n, nnz, h0;
    const i32 *nrp, *nsplit, *ncol, *mirror, *hstart;
    const u32 *ndeg, *order;
    const i64 *wlight, *wheavy;
    const int4 *vmeta;
    const int2 *hseg;
    const i32 *lbeg;
    const i32 *dslot;
};
enum { VM_BEGIN = 0, VM_NSPLIT = 1, VM_END = 2, VM_HSTART = 3 };
inline i32 vmeta_at(const DevGraph &g, i32 v, int f) { return reinterpret_cast<const i32 *>(g.vmeta)[4 * (i64)v + f]; }
#define QS 8
template <int W> inline i64 group_sum64(i64) { abort(); }
inline int row_incl_sum(int) { abort(); }
#include EMU_INC

// one workgroup of nt threads running fn
static void run_block(int nt, size_t dyn_bytes, const std::function<void()> &fn) {
    EmuBlock b;
    b.nt = nt;
    b.bar = new std::barrier<>(nt);
    for (int w = 0; w < nt / WAVE; w++) b.wbar.push_back(new std::barrier<>(WAVE));
    b.xch.assign((size_t)nt, 0);
    b.seqs.assign((size_t)(nt / WAVE), EmuSeqStore{});
    b.dyn = dyn_bytes ? (char *)calloc(dyn_bytes, 1) : nullptr;
    std::vector<std::thread> th;
    for (int t = 0; t < nt; t++)
        th.emplace_back([&, t]() {
            threadIdx.x = t; blockIdx.x = 0; gridDim.x = 1; blockDim.x = nt;
            emu_blk = &b;
            fn();
        });
    for (auto &x : th) x.join();
    for (auto &kv : b.shared) free(kv.second);
    free(b.dyn);
    delete b.bar;
    for (auto *w : b.wbar) delete w;
}

int main(int argc, char **argv) {
    FILE *f = fopen(argv[1], "rb");
    i32 n; i64 nnz;
    fread(&n, 4, 1, f); fread(&nnz, 8, 1, f);
    std::vector<i64> rp(n + 1); std::vector<i32> col(nnz);
    fread(rp.data(), 8, n + 1, f); fread(col.data(), 4, nnz, f); fclose(f);
    const int heavy_k = atoi(argv[2]);
    std::vector<i32> deg(n), order(n), perm(n);
    for (int v = 0; v < n; v++) deg[v] = (i32)(rp[v + 1] - rp[v]);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return deg[a] < deg[b]; });
    for (int y = 0; y < n; y++) perm[order[y]] = y;
    const i32 h0 = n > heavy_k ? n - heavy_k : 0;
    std::vector<i32> nrp(n + 1), nsplit(n), hstart(n), ncol(nnz + 64), mirror(nnz + 64, -1), lbeg(nnz + 64), dslot(nnz + 64);
    std::vector<int2> hseg(nnz + 64);
    std::vector<int4> vmeta(n);
    std::vector<i64> wl(n), wh(n);
    std::vector<u32> ndeg(n);
    nrp[0] = 0;
    for (int y = 0; y < n; y++) {
        int x = order[y];
        std::vector<i32> lo, up;
        for (i64 s = rp[x]; s < rp[x + 1]; s++) { i32 b = perm[col[s]]; (b < y ? lo : up).push_back(b); }
        std::sort(lo.begin(), lo.end()); std::sort(up.begin(), up.end());
        i32 p = nrp[y];
        for (i32 b : lo) ncol[p++] = b;
        nsplit[y] = p;
        for (i32 b : up) ncol[p++] = b;
        nrp[y + 1] = p;
        ndeg[y] = deg[x];
    }
    for (int y = 0; y < n; y++) {
        i32 hs = nrp[y + 1];
        for (i32 s = nsplit[y]; s < nrp[y + 1]; s++) if (ncol[s] >= h0) { hs = s; break; }
        hstart[y] = hs;
        vmeta[y] = int4{nrp[y], nsplit[y], nrp[y + 1], hs};
    }
    for (int y = 0; y < n; y++) {
        i64 a = 0, h = 0;
        for (i32 s = nrp[y]; s < nrp[y + 1]; s++) {
            i32 b = ncol[s];
            const int4 vb = vmeta[b];
            dslot[s] = vb.z - vb.x;
            if (s < nsplit[y]) {
                i32 m = (i32)(std::lower_bound(ncol.begin() + vb.y, ncol.begin() + vb.z, y) - ncol.begin());
                mirror[s] = m; lbeg[s] = vb.x; a += m - vb.x;
                i32 st = (y >= h0) ? std::min(m + 1, vb.z) : vb.w;
                hseg[s] = int2{st, vb.z}; h += vb.z - st;
            } else {
                hseg[s] = int2{vb.w, vb.z}; h += vb.z - vb.w;
            }
        }
        wl[y] = (y < h0) ? a : 0; wh[y] = h;
    }
    DevGraph g{n, (i32)nnz, h0, nrp.data(), nsplit.data(), ncol.data(), mirror.data(), hstart.data(), ndeg.data(),
               (const u32 *)order.data(), wl.data(), wh.data(), vmeta.data(), hseg.data(), lbeg.data(), dslot.data()};
    // classes, as k_classify with the default bounds
    const i64 ql_wave = 512, ql_block = 8192, ql_split = 2048, qh_wave = 512, qh_block = 2048;
    std::vector<std::vector<i32>> lists(WC_COUNT);
    for (int y = n - 1; y >= 0; y--) {
        const i32 d = nrp[y + 1] - nrp[y];
        if (wl[y] > 0) lists[wl[y] <= ql_wave ? WC_QL_WAVE : (wl[y] <= ql_block ? WC_QL_BLOCK : WC_QL_GLOBAL)].push_back(y);
        if (wh[y] > 0)
            lists[d >= 65536 ? WC_QH_GLOBAL : (wh[y] <= qh_wave ? WC_QH_WAVE : (wh[y] <= qh_block ? WC_QH_BLOCK : WC_QH_DENSE))].push_back(y);
    }
    GraphStats st{};
    for (int c = 0; c < WC_COUNT; c++) { st.cnt[c] = (int)lists[c].size(); lists[c].push_back(-7); }
    printf("n=%d nnz=%lld h0=%d classes: qlw %d qlb %d qlg %d qhw %d qhb %d qhd %d qhg %d\n", n, (long long)nnz, h0,
           st.cnt[WC_QL_WAVE], st.cnt[WC_QL_BLOCK], st.cnt[WC_QL_GLOBAL], st.cnt[WC_QH_WAVE], st.cnt[WC_QH_BLOCK],
           st.cnt[WC_QH_DENSE], st.cnt[WC_QH_GLOBAL]);
    if (st.cnt[WC_QL_GLOBAL] || st.cnt[WC_QH_GLOBAL]) { printf("global-class items not emulated\n"); return 2; }
    std::vector<i64> Q(n, 0);
    const i32 K = n - h0;
    std::vector<i64> part((size_t)QH_PART_ROWS * (K > 0 ? K : 1), 0);
    auto pow2 = [](i64 w) { int h = 64; while ((i64)h < 2 * w) h <<= 1; return h; };
    {
        const int hcw = pow2(ql_wave);
        run_block(256, 4 * qlw_wave_bytes(hcw), [&]() { k_q_wave<Q_LIGHT>(g, lists[WC_QL_WAVE].data(), &st, WC_QL_WAVE, Q.data(), hcw); });
        i64 lo = -1, hi = std::min(ql_split, ql_block);
        while (lo < ql_block && hi > 0) {
            const int hcb = pow2(hi);
            run_block(QLB_NT, qlb_bytes(hcb), [&]() { k_q_block<Q_LIGHT>(g, lists[WC_QL_BLOCK].data(), &st, WC_QL_BLOCK, Q.data(), hcb, lo, hi); });
            lo = hi; hi = std::min(2 * hi, ql_block);
        }
    }
    if (K > 0) {
        const int hcw = pow2(qh_wave);
        run_block(256, 4 * qhw_wave_bytes(hcw), [&]() { k_qh_wave(g, lists[WC_QH_WAVE].data(), &st, Q.data(), part.data(), K, hcw); });
        int hcb = 64;
        while ((i64)hcb < 2 * qh_block && hcb < QHB_HC) hcb <<= 1;
        run_block(QHB_NT, (size_t)hcb * 4, [&]() { k_qh_block(g, lists[WC_QH_BLOCK].data(), &st, Q.data(), part.data(), K, hcb); });
        run_block(QD_NT, 0, [&]() { k_q_dense(g, lists[WC_QH_DENSE].data(), &st, Q.data(), part.data(), K); });
        for (int i = 0; i < K; i++) { i64 s = 0; for (int r = 0; r < QH_PART_ROWS; r++) s += part[(size_t)r * K + i]; Q[h0 + i] += s; }
    }
    // direct count
    std::vector<i64> R(n, 0);
    std::vector<i32> cnt(n, 0);
    auto item = [&](i32 x, bool light) {
        const i32 s0 = nrp[x], s1 = light ? nsplit[x] : nrp[x + 1];
        std::vector<i32> touched;
        for (i32 s = s0; s < s1; s++) {
            i32 b0 = light ? lbeg[s] : hseg[s].x, b1 = light ? mirror[s] : hseg[s].y;
            for (i32 p = b0; p < b1; p++) { if (cnt[ncol[p]]++ == 0) touched.push_back(ncol[p]); }
        }
        for (i32 k : touched) { i64 c = cnt[k]; R[x] += c * (c - 1) / 2; R[k] += c * (c - 1) / 2; }
        for (i32 s = s0; s < s1; s++) {
            i32 b0 = light ? lbeg[s] : hseg[s].x, b1 = light ? mirror[s] : hseg[s].y;
            for (i32 p = b0; p < b1; p++) R[ncol[s]] += cnt[ncol[p]] - 1;
        }
        for (i32 k : touched) cnt[k] = 0;
    };
    for (int y = 0; y < n; y++) { if (wl[y] > 0) item(y, true); if (wh[y] > 0) item(y, false); }
    int bad = 0;
    for (int y = 0; y < n; y++) if (Q[y] != R[y]) { if (bad < 10) printf("vertex %d: emulated %lld direct %lld\n", y, (long long)Q[y], (long long)R[y]); bad++; }
    printf("%s: %d vertices differ, sum emulated %lld direct %lld\n", bad ? "MISMATCH" : "ok", bad,
           (long long)std::accumulate(Q.begin(), Q.end(), (i64)0), (long long)std::accumulate(R.begin(), R.end(), (i64)0));
    return bad ? 1 : 0;
}
