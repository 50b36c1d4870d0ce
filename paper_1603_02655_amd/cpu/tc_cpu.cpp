// Multicore CPU census: the thesis's host variant (section v0.7: canonical
// dyads split into task queues of equal |N(u)| + |N(v)| - 2, one local census
// per thread, summed after the join) as a tuned baseline for context.  It is
// not a fallback of the GPU library and shares no code with it or with the
// test oracle.
//
// Per canonical dyad (u, v), u < v, with f = IsEdge(u,v) + 2 IsEdge(v,u)
// (section "Triad Census Algorithm", TriadCode with the pre-computed dyad type
// of v0.4): the third vertices joined to only one of u, v are counted from
// per-row prefix counts of the direction types, and one merge of the two
// sorted neighbour rows finds the shared ones, whose code moves a count from
// the one-sided class to the full class.  Rows hold (w << 2) | f entries.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

#include "tc_cpu.h"

namespace {

// 64 -> 16 class map, from the class definitions (MAN digits and the D/U/C/T
// letters; codes: bit 1 u->v, 2 v->u, 4 u->w, 8 w->u, 16 v->w, 32 w->v).
struct class_map {
    uint8_t t[64];
    class_map() {
        for (int c = 0; c < 64; ++c) t[c] = classify(c);
    }
    static bool arc(int c, int x, int y) {
        static const int bit[3][3] = {{0, 1, 4}, {2, 0, 16}, {8, 32, 0}};
        return x != y && (c & bit[x][y]) != 0;
    }
    static uint8_t classify(int c) {
        int mut = 0, asym = 0;
        const int pr[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (auto& p : pr) {
            bool a = arc(c, p[0], p[1]), b = arc(c, p[1], p[0]);
            mut += a && b;
            asym += a != b;
        }
        int outd[3] = {0, 0, 0}, ind[3] = {0, 0, 0};
        for (int x = 0; x < 3; ++x)
            for (int y = 0; y < 3; ++y)
                if (arc(c, x, y) && !arc(c, y, x)) { ++outd[x]; ++ind[y]; }
        auto any = [&](const int* d, int k) { return d[0] == k || d[1] == k || d[2] == k; };
        if (mut == 0 && asym == 0) return 0;                                  // 003
        if (mut == 0 && asym == 1) return 1;                                  // 012
        if (mut == 1 && asym == 0) return 2;                                  // 102
        if (mut == 0 && asym == 2) return any(outd, 2) ? 3 : any(ind, 2) ? 4 : 5;  // 021D U C
        if (mut == 1 && asym == 1) {
            // 111D: the asymmetric arc enters the mutual dyad; 111U: it leaves it
            for (int x = 0; x < 3; ++x)
                for (int y = 0; y < 3; ++y)
                    if (arc(c, x, y) && !arc(c, y, x)) {
                        int z = 3 - x - y;
                        return (arc(c, y, z) && arc(c, z, y)) ? 6 : 7;
                    }
        }
        if (mut == 0 && asym == 3) return any(outd, 2) ? 8 : 9;              // 030T, 030C
        if (mut == 2 && asym == 0) return 10;                                 // 201
        if (mut == 1 && asym == 2) return any(outd, 2) ? 11 : any(ind, 2) ? 12 : 13;  // 120D U C
        if (mut == 2 && asym == 1) return 14;                                 // 210
        return 15;                                                            // 300
    }
};

struct csr {
    int32_t n = 0;
    std::vector<uint64_t> ptr;    // n + 1
    std::vector<uint32_t> nbr;    // (w << 2) | f, f relative to the row's owner
    std::vector<uint64_t> cnt_hi; // per entry: (#out << 32) | #in over the entries after it in its row
};

bool build(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, csr& g) {
    std::vector<uint64_t> keys;
    keys.reserve(2 * (size_t)m);
    for (int64_t i = 0; i < m; ++i) {
        const int32_t a = src[i], b = dst[i];
        if (a < 0 || b < 0 || a >= n || b >= n) return false;
        if (a == b) continue;
        keys.push_back(((uint64_t)a << 34) | ((uint64_t)b << 2) | 1u);
        keys.push_back(((uint64_t)b << 34) | ((uint64_t)a << 2) | 2u);
    }
    std::sort(keys.begin(), keys.end());
    g.n = n;
    g.ptr.assign((size_t)n + 1, 0);
    g.nbr.clear();
    g.nbr.reserve(keys.size());
    for (size_t i = 0; i < keys.size();) {
        const uint64_t k = keys[i] >> 2;
        uint32_t f = 0;
        while (i < keys.size() && (keys[i] >> 2) == k) f |= (uint32_t)(keys[i++] & 3u);
        const uint32_t owner = (uint32_t)(k >> 32), w = (uint32_t)(k & 0xffffffffu);
        g.ptr[owner + 1]++;
        g.nbr.push_back((w << 2) | f);
    }
    for (int32_t u = 0; u < n; ++u) g.ptr[u + 1] += g.ptr[u];
    // typed counts of the entries after each entry in its row
    g.cnt_hi.assign(g.nbr.size(), 0);
    for (int32_t u = 0; u < n; ++u) {
        uint64_t out = 0, in = 0;
        for (uint64_t p = g.ptr[u + 1]; p-- > g.ptr[u];) {
            g.cnt_hi[p] = (out << 32) | in;
            out += g.nbr[p] & 1u;
            in += (g.nbr[p] >> 1) & 1u;
        }
    }
    return true;
}

void census_rows(const csr& g, const class_map& T, int32_t u0, int32_t u1, uint64_t c[16]) {
    const uint64_t n = (uint64_t)g.n;
    const uint32_t* nb = g.nbr.data();
    for (int32_t u = u0; u < u1; ++u) {
        const uint64_t bu = g.ptr[u], eu = g.ptr[u + 1], du = eu - bu;
        for (uint64_t iv = bu; iv < eu; ++iv) {
            const uint32_t v = nb[iv] >> 2;
            if (v <= (uint32_t)u) continue;
            const uint32_t f = nb[iv] & 3u;
            const uint64_t bv = g.ptr[v], ev = g.ptr[v + 1], dv = ev - bv;
            c[T.t[f]] += n - du - dv;
            // N(u) above v, N(v) above u, by direction type (out only, in only, mutual)
            const uint64_t pa = g.cnt_hi[iv];
            const uint64_t a_out = pa >> 32, a_in = pa & 0xffffffffu, a_tot = eu - iv - 1;
            const uint64_t a3 = a_out + a_in - a_tot;
            c[T.t[f | 4u]] += a_out - a3;
            c[T.t[f | 8u]] += a_in - a3;
            c[T.t[f | 12u]] += a3;
            // position of u in N(v): rows are sorted, binary search
            const uint32_t* rv = nb + bv;
            const uint64_t iu = bv + (uint64_t)(std::lower_bound(rv, rv + dv, (uint32_t)u << 2) - rv);
            const uint64_t pb = g.cnt_hi[iu];
            const uint64_t b_out = pb >> 32, b_in = pb & 0xffffffffu, b_tot = ev - iu - 1;
            const uint64_t b3 = b_out + b_in - b_tot;
            c[T.t[f | 16u]] += b_out - b3;
            c[T.t[f | 32u]] += b_in - b3;
            c[T.t[f | 48u]] += b3;
            // shared neighbours
            uint64_t i = bu, j = bv;
            while (i < eu && j < ev) {
                const uint32_t a = nb[i] >> 2, b = nb[j] >> 2;
                if (a < b) { ++i; continue; }
                if (b < a) { ++j; continue; }
                const uint32_t fa = nb[i] & 3u, fb = nb[j] & 3u, w = a;
                c[T.t[f]] += 1;                                   // |S| is one smaller
                if (w > v) {
                    c[T.t[f | (fa << 2) | (fb << 4)]] += 1;
                    c[T.t[f | (fa << 2)]] -= 1;
                }
                if (w > (uint32_t)u) c[T.t[f | (fb << 4)]] -= 1;
                ++i;
                ++j;
            }
        }
    }
}

}  // namespace

extern "C" int tc_cpu_census(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, int32_t threads,
                             uint64_t counts[16], double* census_seconds) {
    if (n < 0 || m < 0 || (m > 0 && (!src || !dst)) || !counts) return -1;
    static const class_map T;
    csr g;
    if (!build(n, m, src, dst, g)) return -1;
    if (threads <= 0) threads = (int32_t)std::max(1u, std::thread::hardware_concurrency());
    // task queues: runs of rows of about equal dyad work sum(|N(u)| + |N(v)|),
    // handed out dynamically, many more runs than threads
    std::vector<double> work((size_t)n + 1, 0.0);
    for (int32_t u = 0; u < n; ++u) {
        double s = 0;
        for (uint64_t p = g.ptr[u]; p < g.ptr[u + 1]; ++p) {
            const uint32_t v = g.nbr[p] >> 2;
            if (v > (uint32_t)u) s += (double)(g.ptr[u + 1] - g.ptr[u] + g.ptr[v + 1] - g.ptr[v]);
        }
        work[u + 1] = work[u] + s + 1.0;
    }
    const int64_t runs = std::max<int64_t>(1, (int64_t)threads * 64);
    std::vector<int32_t> cut((size_t)runs + 1, n);
    cut[0] = 0;
    for (int64_t r = 1; r < runs; ++r) {
        const double target = work[n] * (double)r / (double)runs;
        cut[r] = (int32_t)(std::lower_bound(work.begin(), work.end(), target) - work.begin());
        if (cut[r] > n) cut[r] = n;
        if (cut[r] < cut[r - 1]) cut[r] = cut[r - 1];
    }
    std::atomic<int64_t> next{0};
    std::vector<std::array<uint64_t, 16>> local((size_t)threads);
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<std::thread> pool;
    for (int32_t t = 0; t < threads; ++t)
        pool.emplace_back([&, t]() {
            uint64_t c[16] = {0};
            for (int64_t r; (r = next.fetch_add(1)) < runs;) census_rows(g, T, cut[r], cut[r + 1], c);
            std::memcpy(local[t].data(), c, sizeof(c));
        });
    for (auto& th : pool) th.join();
    const auto t1 = std::chrono::steady_clock::now();
    if (census_seconds) *census_seconds = std::chrono::duration<double>(t1 - t0).count();
    typedef unsigned __int128 u128;
    uint64_t c[16] = {0};
    for (auto& l : local)
        for (int k = 0; k < 16; ++k) c[k] += l[k];
    const u128 total = n >= 3 ? (u128)n * (u128)(n - 1) * (u128)(n - 2) / 6 : 0;
    u128 sum = 0;
    for (int k = 1; k < 16; ++k) sum += c[k];
    c[0] = (uint64_t)(total - sum);
    std::memcpy(counts, c, sizeof(c));
    return 0;
}
