// Census kernels: one canonical dyad (u, v), u < v, per task, following the
// subquadratic census (section "Triad Census Algorithm", figure "Subquadratic
// Triad Census Algorithm") with the pre-computed dyad type of the v0.4 change.
//
// Per dyad with f = IsEdge(u,v) + 2 IsEdge(v,u):
//   * dyadic triads:  n - |S| - 2 = n - |N(u)| - |N(v)| + |N(u) ^ N(v)| go to
//     class 102 if f == 3, else 012;
//   * a third vertex w in S is counted (the canonical condition
//     v < w  or  (u < w < v and w not adjacent to u)) exactly when
//       w in N(u) and w > v            (code f | f_uw << 2 | f_vw << 4), or
//       w in N(v) \ N(u) and w > u     (code f | f_vw << 4);
//   * classes come from the 64 -> 16 table.
// Non-shared third vertices never need to be visited one by one: the number
// of entries of each direction type in a row range is a difference of the
// row's prefix counts (tpre), so a dyad adds those totals once and the merge of
// N(u) and N(v) only has to find the shared vertices, each of which moves one
// count from its single-list class to its full-code class.
//
// Three execution modes over the degree buckets (key |N(u)| + |N(v)| - 2):
//   lane  : one lane per dyad, two-pointer merge of the two rows;
//   wave  : one 64-lane wavefront per dyad, merge path over LDS-staged tiles;
//   group : one 256-lane workgroup per dyad, merge path over larger tiles.
// Counts accumulate in 64-bit LDS bins (private per lane in the lane mode, per
// wavefront elsewhere); each workgroup adds its 16 sums to the graph's
// accumulators with one 64-bit global atomic per class when it finishes.
#include "tc_census.h"

namespace tc {

namespace {

__constant__ uint8_t c_table[64];

// ---- class histograms in LDS ------------------------------------------------
// lane_bins: one private 16-bin row per lane (no contention; used where every
// lane works on its own dyad).  wave_bins: 16 bins per wavefront updated with
// LDS atomics (used where a group shares a dyad and only shared neighbours and
// one lane's per-dyad totals are added).
template <int B>
struct lane_bins {
    static constexpr int kWords = kNumClasses * B;
    unsigned long long* bins;
    __device__ inline void add(uint32_t cls, unsigned long long x) {
        atomicAdd(&bins[cls * B + threadIdx.x], x);
    }
    __device__ inline void clear() {
        for (int i = threadIdx.x; i < kWords; i += B) bins[i] = 0;
    }
    __device__ inline void flush(unsigned long long* acc) {
        __syncthreads();
        const int lane = __lane_id(), wid = threadIdx.x >> 6;
        for (int cls = wid; cls < kNumClasses; cls += B / 64) {
            unsigned long long s = 0;
            for (int i = lane; i < B; i += 64) s += bins[cls * B + i];
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
            if (lane == 0 && s != 0) atomicAdd(&acc[cls], s);
        }
    }
};

template <int B>
struct wave_bins {
    static constexpr int kWords = kNumClasses * (B / 64);
    unsigned long long* bins;
    __device__ inline void add(uint32_t cls, unsigned long long x) {
        atomicAdd(&bins[(threadIdx.x >> 6) * kNumClasses + cls], x);
    }
    __device__ inline void clear() {
        for (int i = threadIdx.x; i < kWords; i += B) bins[i] = 0;
    }
    __device__ inline void flush(unsigned long long* acc) {
        __syncthreads();
        if (threadIdx.x < kNumClasses) {
            unsigned long long s = 0;
            for (int w = 0; w < B / 64; ++w) s += bins[w * kNumClasses + threadIdx.x];
            if (s != 0) atomicAdd(&acc[threadIdx.x], s);
        }
    }
};

// Per-dyad totals that do not depend on the shared vertices: the dyadic base
// n - |N(u)| - |N(v)| and, per direction type t (1 out, 2 in, 3 mutual), the
// entries of N(u) above v and of N(v) above u, from the prefix counts.
struct dyad_totals {
    uint64_t pa0, pa1, pb0, pb1;   // tpre at (iv+1, eu) and (iu+1, ev)
};

__device__ inline dyad_totals load_totals(const dyad_rec& r, const uint64_t* __restrict__ tpre) {
    return dyad_totals{tpre[r.iv + 1], tpre[r.eu], tpre[r.iu + 1], tpre[r.ev]};
}

template <class H>
__device__ inline void add_totals(const dyad_rec& r, const dyad_totals& t, uint64_t n, const uint8_t* T, H& h) {
    const uint32_t f = r.vf & 3u;
    const uint64_t du = r.eu - r.bu, dv = r.ev - r.bv;
    h.add(f == 3u ? 2u : 1u, (unsigned long long)(n - du - dv));
    uint64_t pa = t.pa1 - t.pa0;                       // N(u) entries w > v
    uint64_t a_tot = r.eu - r.iv - 1, a_out = pa & 0xffffffffull, a_in = pa >> 32;
    uint64_t a3 = a_out + a_in - a_tot;
    h.add(T[f | 4u], a_out - a3);
    h.add(T[f | 8u], a_in - a3);
    h.add(T[f | 12u], a3);
    uint64_t pb = t.pb1 - t.pb0;                       // N(v) entries w > u
    uint64_t b_tot = r.ev - r.iu - 1, b_out = pb & 0xffffffffull, b_in = pb >> 32;
    uint64_t b3 = b_out + b_in - b_tot;
    h.add(T[f | 16u], b_out - b3);
    h.add(T[f | 32u], b_in - b3);
    h.add(T[f | 48u], b3);
}

// A vertex w adjacent to both u (entry flags fa) and v (flags fb).
template <class H>
__device__ inline void on_common(uint32_t w, uint32_t fa, uint32_t fb, uint32_t u, uint32_t v, uint32_t f,
                                 const uint8_t* T, H& h) {
    h.add(f == 3u ? 2u : 1u, 1ull);                       // |S| is one smaller
    if (w > v) {                                          // counted with its full code
        h.add(T[f | (fa << 2) | (fb << 4)], 1ull);
        h.add(T[f | (fa << 2)], ~0ull);                   // not a u-only vertex
    }
    if (w > u) h.add(T[f | (fb << 4)], ~0ull);            // not a v-only vertex
}

__device__ inline dyad_rec load_rec(const dyad_rec* p) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
    uint4 a = q[0], b = q[1];
    dyad_rec r;
    r.bu = a.x; r.eu = a.y; r.bv = a.z; r.ev = a.w;
    r.iv = b.x; r.iu = b.y; r.u = b.z; r.vf = b.w;
    return r;
}

// Entries are (w << 2) | f with w < 2^23, so the all-ones word never occurs
// and serves as the end-of-list sentinel.  Comparing vertices of two entries:
//   w(a) <= w(b)  <=>  a <= (b | 3),      w(a) == w(b)  <=>  (a ^ b) < 4.
constexpr uint32_t kSentinel = 0xffffffffu;

// ---------------------------------------------------------------- lane ----
// One lane per dyad: a two-pointer merge of rows u and v read from global
// memory (L1/L2 resident for the short rows of this bucket).
constexpr int kLaneB = 256;

template <class H>
__device__ inline void lane_dyad(const dyad_rec& r, const uint32_t* __restrict__ nbr, const uint64_t* __restrict__ tpre,
                                 uint64_t n, const uint8_t* T, H& h) {
    const dyad_totals t = load_totals(r, tpre);
    const uint32_t u = r.u, v = r.vf >> 2, f = r.vf & 3u;
    uint32_t i = r.bu, j = r.bv;
    // rows are never empty: v is in row u and u is in row v
    uint32_t a = nbr[i], b = nbr[j];
    for (;;) {
        if ((a ^ b) < 4u) on_common(a >> 2, a & 3u, b & 3u, u, v, f, T, h);
        if (a <= (b | 3u)) {
            if (++i >= r.eu) break;
            a = nbr[i];
        } else {
            if (++j >= r.ev) break;
            b = nbr[j];
        }
    }
    add_totals(r, t, n, T, h);
}

__global__ __launch_bounds__(kLaneB) void k_census_lane(census_args L) {
    extern __shared__ unsigned long long lds[];
    __shared__ uint8_t T[64];
    if (threadIdx.x < 64) T[threadIdx.x] = c_table[threadIdx.x];
    lane_bins<kLaneB> h{lds};
    h.clear();
    __syncthreads();
    for (uint64_t d = (uint64_t)blockIdx.x * kLaneB + threadIdx.x; d < L.count;
         d += (uint64_t)gridDim.x * kLaneB)
        lane_dyad(load_rec(L.dyads + d), L.nbr, L.tpre, L.n, T, h);
    h.flush(L.acc);
}

// ---------------------------------------------------------- merge path ----
// Group-cooperative intersection of rows [bu, eu) and [bv, ev) in rounds.  A
// round stages the next TW entries of each row in LDS (followed by a
// sentinel), produces the first min(TW, na + nb) outputs of the merged order
// (ties: the N(u) copy first), and lane l handles outputs [l*PER, (l+1)*PER)
// after locating its start on the merge path by binary search (co-rank).  A
// shared vertex is seen when its N(u) copy is taken while the N(v) head holds
// the same vertex.  The lane that produces the round's last output publishes
// how many N(u) entries the round consumed.
__device__ inline uint32_t co_rank(const uint32_t* sA, uint32_t na, const uint32_t* sB, uint32_t nb, uint32_t d) {
    uint32_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (sA[mid - 1] <= (sB[d - mid] | 3u)) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Synchronisation of the group that shares a dyad: the whole workgroup, or a
// single wavefront (whose lanes run in lockstep, LDS accesses in order; the
// fences keep the compiler from moving LDS accesses across the point).
struct block_sync {
    __device__ inline void operator()() const { __syncthreads(); }
};
struct wave_sync {
    __device__ inline void operator()() const {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

template <int G, int TW, class Sync, class H>
__device__ inline void merge_path(const dyad_rec& r, const uint32_t* __restrict__ nbr, uint32_t* sA, uint32_t* sB,
                                  uint32_t* s_xt, uint32_t lane, const uint8_t* T, H& h) {
    constexpr uint32_t PER = TW / G;
    static_assert(TW % G == 0, "tile is a multiple of the group");
    const Sync sync{};
    const uint32_t u = r.u, v = r.vf >> 2, f = r.vf & 3u;
    const uint32_t la = r.eu - r.bu, lb = r.ev - r.bv;
    uint32_t a_pos = 0, b_pos = 0;
    while (a_pos < la && b_pos < lb) {
        const uint32_t na = min((uint32_t)TW, la - a_pos), nb = min((uint32_t)TW, lb - b_pos);
        uint32_t ra[PER], rb[PER];
#pragma unroll
        for (uint32_t t = 0; t < PER; ++t) {
            const uint32_t k = lane + t * G;
            ra[t] = k < na ? nbr[r.bu + a_pos + k] : kSentinel;
            rb[t] = k < nb ? nbr[r.bv + b_pos + k] : kSentinel;
        }
#pragma unroll
        for (uint32_t t = 0; t < PER; ++t) {
            sA[lane + t * G] = ra[t];
            sB[lane + t * G] = rb[t];
        }
        if (lane == 0) {
            sA[TW] = kSentinel;
            sB[TW] = kSentinel;
        }
        sync();
        const uint32_t total = min((uint32_t)TW, na + nb);
        const uint32_t d0 = lane * PER;
        if (d0 < total) {
            const uint32_t steps = min(PER, total - d0);
            uint32_t i = co_rank(sA, na, sB, nb, d0);
            uint32_t j = d0 - i;
            uint32_t a = sA[i], b = sB[j];
#pragma unroll
            for (uint32_t t = 0; t < PER; ++t) {
                if (t < steps) {
                    if ((a ^ b) < 4u) on_common(a >> 2, a & 3u, b & 3u, u, v, f, T, h);
                    const bool ta = a <= (b | 3u);
                    i += ta ? 1u : 0u;
                    j += ta ? 0u : 1u;
                    const uint32_t x = ta ? sA[i] : sB[j];
                    a = ta ? x : a;
                    b = ta ? b : x;
                }
            }
            if (d0 + steps == total) *s_xt = i;
        }
        sync();
        const uint32_t xt = *s_xt;
        a_pos += xt;
        b_pos += total - xt;
    }
}

// ------------------------------------------------------ work distribution ----
// Dyads are handed out in chunks of CH through eight counters, one per XCD
// (workgroup b runs on XCD b % 8 on this part), so that the atomics stay in
// one L2: counter x hands out the chunk indices x, x + 8, x + 16, ...
constexpr int kXcds = 8;

__device__ inline uint32_t take_chunk(unsigned int* ctr, uint32_t xcd) {
    return xcd + kXcds * atomicAdd(&ctr[xcd], 1u);
}

// ---------------------------------------------------------------- wave ----
constexpr int kWaveB = 64;
constexpr int kWaveTile = 1024;
constexpr uint32_t kWaveChunk = 16;

__global__ __launch_bounds__(kWaveB) void k_census_wave(census_args L, unsigned int* ctr) {
    __shared__ unsigned long long bins[wave_bins<kWaveB>::kWords];
    __shared__ uint8_t T[64];
    __shared__ uint32_t sA[kWaveTile + 1], sB[kWaveTile + 1];
    __shared__ uint32_t s_xt;
    T[threadIdx.x] = c_table[threadIdx.x];
    wave_bins<kWaveB> h{bins};
    h.clear();
    __syncthreads();
    const uint32_t xcd = blockIdx.x % kXcds;
    uint32_t c = 0;
    if (threadIdx.x == 0) c = take_chunk(ctr, xcd);
    c = __shfl(c, 0, 64);
    while ((uint64_t)c * kWaveChunk < L.count) {
        uint32_t cn = 0;
        if (threadIdx.x == 0) cn = take_chunk(ctr, xcd);      // next chunk, fetched early
        const uint32_t end = min((uint32_t)L.count, (c + 1) * kWaveChunk);
        for (uint32_t d = c * kWaveChunk; d < end; ++d) {
            const dyad_rec r = load_rec(L.dyads + d);
            dyad_totals t{};
            if (threadIdx.x == 0) t = load_totals(r, L.tpre);
            merge_path<kWaveB, kWaveTile, block_sync>(r, L.nbr, sA, sB, &s_xt, threadIdx.x, T, h);
            if (threadIdx.x == 0) add_totals(r, t, L.n, T, h);
        }
        c = __shfl(cn, 0, 64);
    }
    h.flush(L.acc);
}

// --------------------------------------------------------------- group ----
constexpr int kGroupB = 256;
constexpr int kGroupTile = 4096;
constexpr uint32_t kGroupChunk = 2;

__global__ __launch_bounds__(kGroupB) void k_census_group(census_args L, unsigned int* ctr) {
    __shared__ unsigned long long bins[wave_bins<kGroupB>::kWords];
    __shared__ uint8_t T[64];
    __shared__ uint32_t sA[kGroupTile + 1], sB[kGroupTile + 1];
    __shared__ uint32_t s_xt, s_next;
    if (threadIdx.x < 64) T[threadIdx.x] = c_table[threadIdx.x];
    wave_bins<kGroupB> h{bins};
    h.clear();
    const uint32_t xcd = blockIdx.x % kXcds;
    if (threadIdx.x == 0) s_next = take_chunk(ctr, xcd);
    __syncthreads();
    uint32_t c = s_next;
    __syncthreads();
    while ((uint64_t)c * kGroupChunk < L.count) {
        if (threadIdx.x == 0) s_next = take_chunk(ctr, xcd);  // next chunk, fetched early
        const uint32_t end = min((uint32_t)L.count, (c + 1) * kGroupChunk);
        for (uint32_t d = c * kGroupChunk; d < end; ++d) {
            const dyad_rec r = load_rec(L.dyads + d);
            dyad_totals t{};
            if (threadIdx.x == 0) t = load_totals(r, L.tpre);
            merge_path<kGroupB, kGroupTile, block_sync>(r, L.nbr, sA, sB, &s_xt, threadIdx.x, T, h);
            if (threadIdx.x == 0) add_totals(r, t, L.n, T, h);
        }
        __syncthreads();
        c = s_next;
        __syncthreads();
    }
    h.flush(L.acc);
}


// --------------------------------------------------------------- batch ----
// One persistent launch over the work items of many resident graphs.  A
// workgroup takes items one at a time (per-XCD counters); an item is a slice of
// one graph's bucket: up to 256 lane-mode dyads (one per thread), up to
// 4 * kBatchWavePerItem wave-mode dyads (wavefront w takes every fourth), or one
// group-mode dyad.  Counts go to per-lane bins that are flushed into the
// graph's 16 accumulators whenever the workgroup moves to another graph.
constexpr int kBatchB = 256;
constexpr int kBatchWaveTile = 512;
constexpr int kBatchGroupTile = 2048;
constexpr int kBatchTileWords = (4 * 2 * (kBatchWaveTile + 1) > 2 * (kBatchGroupTile + 1))
                                    ? 4 * 2 * (kBatchWaveTile + 1) : 2 * (kBatchGroupTile + 1);

__global__ __launch_bounds__(kBatchB) void k_census_batch(const graph_desc* __restrict__ G,
                                                          const work_item* __restrict__ items,
                                                          const uint32_t* __restrict__ num_items,
                                                          unsigned long long* __restrict__ accs,
                                                          unsigned int* __restrict__ ctr) {
    extern __shared__ unsigned long long lds[];
    __shared__ uint8_t T[64];
    __shared__ uint32_t tiles[kBatchTileWords];
    __shared__ uint32_t s_xt[kBatchB / 64], s_next;
    if (threadIdx.x < 64) T[threadIdx.x] = c_table[threadIdx.x];
    lane_bins<kBatchB> h{lds};
    h.clear();
    const uint32_t count = *num_items;
    const uint32_t xcd = blockIdx.x % kXcds;
    const uint32_t tid = threadIdx.x, wid = tid >> 6, lane = tid & 63u;
    uint32_t cur = 0xffffffffu;
    if (tid == 0) s_next = take_chunk(ctr, xcd);
    __syncthreads();
    uint32_t idx = s_next;
    __syncthreads();
    while (idx < count) {
        if (tid == 0) s_next = take_chunk(ctr, xcd);
        const work_item it = items[idx];
        if (it.graph != cur) {
            if (cur != 0xffffffffu) {
                h.flush(accs + (uint64_t)kNumClasses * cur);
                __syncthreads();
                h.clear();
            }
            cur = it.graph;
            __syncthreads();
        }
        const graph_desc g = G[it.graph];
        if (it.kind == kItemLane) {
            const uint32_t d = it.begin + tid;
            if (d < it.end) lane_dyad(load_rec(g.dyads + d), g.nbr, g.tpre, g.n, T, h);
        } else if (it.kind == kItemWave) {
            uint32_t* sA = tiles + wid * 2 * (kBatchWaveTile + 1);
            uint32_t* sB = sA + kBatchWaveTile + 1;
            for (uint32_t d = it.begin + wid; d < it.end; d += kBatchB / 64) {
                const dyad_rec r = load_rec(g.dyads + d);
                dyad_totals t{};
                if (lane == 0) t = load_totals(r, g.tpre);
                merge_path<64, kBatchWaveTile, wave_sync>(r, g.nbr, sA, sB, &s_xt[wid], lane, T, h);
                if (lane == 0) add_totals(r, t, g.n, T, h);
            }
        } else {
            const dyad_rec r = load_rec(g.dyads + it.begin);
            dyad_totals t{};
            if (tid == 0) t = load_totals(r, g.tpre);
            merge_path<kBatchB, kBatchGroupTile, block_sync>(r, g.nbr, tiles, tiles + kBatchGroupTile + 1, &s_xt[0],
                                                              tid, T, h);
            if (tid == 0) add_totals(r, t, g.n, T, h);
        }
        __syncthreads();
        idx = s_next;
        __syncthreads();
    }
    if (cur != 0xffffffffu) h.flush(accs + (uint64_t)kNumClasses * cur);
}

__global__ void k_fill_u64_grid(unsigned long long* p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_zero_u32(unsigned int* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

}  // namespace

hipError_t batch_launch(const graph_desc* descs, const work_item* items, const uint32_t* num_items,
                        unsigned long long* accs, uint64_t acc_words, unsigned int* counters, uint32_t grid,
                        hipStream_t s) {
    uint32_t zb = (uint32_t)std::min<uint64_t>((acc_words + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_u64_grid, dim3(zb ? zb : 1), dim3(256), 0, s, accs, acc_words);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, counters, kXcds);
    hipLaunchKernelGGL(k_census_batch, dim3(grid), dim3(kBatchB), sizeof(unsigned long long) * lane_bins<kBatchB>::kWords,
                       s, descs, items, num_items, accs, counters);
    return hipGetLastError();
}

hipError_t census_upload_table() {
    return hipMemcpyToSymbol(HIP_SYMBOL(c_table), kTable.t, sizeof(kTable.t));
}

hipError_t census_launch(const device_graph& g, const census_slices& sl, unsigned long long* acc,
                         unsigned int* counters, const census_config& cfg, hipStream_t s, hipEvent_t* ev) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, acc, kNumClasses);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, counters, 3 * kXcds);
    for (int b = 0; b < kBuckets; ++b) {
        uint64_t cnt = sl.end[b] > sl.begin[b] ? sl.end[b] - sl.begin[b] : 0;
        if (ev) (void)hipEventRecord(ev[2 * b], s);
        if (cnt > 0) {
            census_args L{g.dyads + sl.begin[b], (uint32_t)cnt, g.nbr, g.tpre, (uint64_t)g.n, acc};
            if (b == 0) {
                uint32_t grid = (uint32_t)std::min<uint64_t>((cnt + kLaneB - 1) / kLaneB, cfg.lane_blocks);
                size_t sh = sizeof(unsigned long long) * lane_bins<kLaneB>::kWords;
                hipLaunchKernelGGL(k_census_lane, dim3(grid), dim3(kLaneB), sh, s, L);
            } else if (b == 1) {
                uint32_t grid = (uint32_t)std::min<uint64_t>(cnt, cfg.wave_blocks);
                hipLaunchKernelGGL(k_census_wave, dim3(grid), dim3(kWaveB), 0, s, L, counters + kXcds);
            } else {
                uint32_t grid = (uint32_t)std::min<uint64_t>(cnt, cfg.group_blocks);
                hipLaunchKernelGGL(k_census_group, dim3(grid), dim3(kGroupB), 0, s, L, counters + 2 * kXcds);
            }
        }
        if (ev) (void)hipEventRecord(ev[2 * b + 1], s);
    }
    return hipGetLastError();
}

}  // namespace tc
