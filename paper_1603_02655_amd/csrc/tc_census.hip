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
// Counts accumulate in per-lane private 64-bit LDS bins; each workgroup adds
// its 16 sums to the graph's accumulators with one 64-bit atomic per class.
#include "tc_census.h"

namespace tc {

namespace {

__constant__ uint8_t c_table[64];

// ---- per-lane private histogram in LDS -----------------------------------
template <int B>
struct lane_hist {
    unsigned long long* bins;   // [16][B]
    int tid;
    __device__ inline void add(uint32_t cls, unsigned long long x) {
        atomicAdd(&bins[cls * B + tid], x);
    }
};

template <int B>
__device__ inline void hist_clear(unsigned long long* bins) {
    for (int i = threadIdx.x; i < kNumClasses * B; i += B) bins[i] = 0;
}

// Reduces the per-lane bins of the block and adds them to the graph accumulators.
template <int B>
__device__ inline void hist_flush(unsigned long long* bins, unsigned long long* acc) {
    __syncthreads();
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    constexpr int W = B / 64;
    for (int cls = wid; cls < kNumClasses; cls += W) {
        unsigned long long s = 0;
        for (int i = lane; i < B; i += 64) s += bins[cls * B + i];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0 && s != 0) atomicAdd(&acc[cls], s);
    }
}

// Totals of one dyad that do not depend on the shared vertices: the dyadic
// base n - |N(u)| - |N(v)| and, per direction type t (1 out, 2 in, 3 mutual),
// the entries of N(u) above v and of N(v) above u.
template <int B>
__device__ inline void dyad_base(const dyad_rec& r, const uint64_t* __restrict__ tpre, uint64_t n,
                                 const uint8_t* T, lane_hist<B>& h) {
    const uint32_t f = r.vf & 3u;
    const uint64_t du = r.eu - r.bu, dv = r.ev - r.bv;
    h.add(f == 3u ? 2u : 1u, (unsigned long long)(n - du - dv));
    // N(u) entries w > v: positions (iv, eu)
    uint64_t pa = tpre[r.eu] - tpre[r.iv + 1];
    uint64_t a_tot = r.eu - r.iv - 1, a_out = pa & 0xffffffffull, a_in = pa >> 32;
    uint64_t a3 = a_out + a_in - a_tot;
    h.add(T[f | 4u], a_out - a3);
    h.add(T[f | 8u], a_in - a3);
    h.add(T[f | 12u], a3);
    // N(v) entries w > u: positions (iu, ev)
    uint64_t pb = tpre[r.ev] - tpre[r.iu + 1];
    uint64_t b_tot = r.ev - r.iu - 1, b_out = pb & 0xffffffffull, b_in = pb >> 32;
    uint64_t b3 = b_out + b_in - b_tot;
    h.add(T[f | 16u], b_out - b3);
    h.add(T[f | 32u], b_in - b3);
    h.add(T[f | 48u], b3);
}

// A vertex w adjacent to both u (entry flags fa) and v (flags fb).
template <int B>
__device__ inline void on_common(uint32_t w, uint32_t fa, uint32_t fb, uint32_t u, uint32_t v, uint32_t f,
                                 const uint8_t* T, lane_hist<B>& h) {
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

// ---------------------------------------------------------------- lane ----
constexpr int kLaneB = 256;

__global__ __launch_bounds__(kLaneB) void k_census_lane(census_args L) {
    extern __shared__ unsigned long long lds[];
    __shared__ uint8_t T[64];
    unsigned long long* bins = lds;
    if (threadIdx.x < 64) T[threadIdx.x] = c_table[threadIdx.x];
    hist_clear<kLaneB>(bins);
    __syncthreads();
    lane_hist<kLaneB> h{bins, (int)threadIdx.x};
    const uint32_t* __restrict__ nbr = L.nbr;
    for (uint64_t d = (uint64_t)blockIdx.x * kLaneB + threadIdx.x; d < L.count;
         d += (uint64_t)gridDim.x * kLaneB) {
        dyad_rec r = load_rec(L.dyads + d);
        dyad_base<kLaneB>(r, L.tpre, L.n, T, h);
        const uint32_t u = r.u, v = r.vf >> 2, f = r.vf & 3u;
        uint32_t i = r.bu, j = r.bv;
        while (i < r.eu && j < r.ev) {
            uint32_t a = nbr[i], b = nbr[j];
            uint32_t wa = a >> 2, wb = b >> 2;
            if (wa == wb) on_common<kLaneB>(wa, a & 3u, b & 3u, u, v, f, T, h);
            i += (wa <= wb);
            j += (wb <= wa);
        }
    }
    hist_flush<kLaneB>(bins, L.acc);
}

// ---------------------------------------------------------- merge path ----
// Group-cooperative intersection of rows [bu, eu) and [bv, ev) in tiles of TW
// entries per row staged in LDS.  Each round produces up to TW outputs of the
// merged order (ties: the N(u) copy first); lane l handles outputs
// [l*TW/G, (l+1)*TW/G) after locating its start by binary search on the merge
// path.  A shared vertex is detected when its N(u) copy is taken while the N(v)
// head holds the same vertex.
__device__ inline uint32_t co_rank(const uint32_t* sA, uint32_t na, const uint32_t* sB, uint32_t nb, uint32_t d) {
    uint32_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if ((sA[mid - 1] >> 2) <= (sB[d - mid] >> 2)) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int G, int TW>
__device__ inline void merge_path(const dyad_rec& r, const uint32_t* __restrict__ nbr, uint32_t* sA, uint32_t* sB,
                                  const uint8_t* T, lane_hist<G>& h) {
    constexpr uint32_t PER = TW / G;
    const uint32_t lane = threadIdx.x;
    const uint32_t u = r.u, v = r.vf >> 2, f = r.vf & 3u;
    const uint32_t la = r.eu - r.bu, lb = r.ev - r.bv;
    uint32_t a_pos = 0, b_pos = 0;
    while (a_pos < la && b_pos < lb) {
        const uint32_t na = min((uint32_t)TW, la - a_pos), nb = min((uint32_t)TW, lb - b_pos);
        for (uint32_t k = lane; k < na; k += G) sA[k] = nbr[r.bu + a_pos + k];
        for (uint32_t k = lane; k < nb; k += G) sB[k] = nbr[r.bv + b_pos + k];
        __syncthreads();
        const uint32_t total = min((uint32_t)TW, na + nb);
        const uint32_t d0 = lane * PER, d1 = min(d0 + PER, total);
        if (d0 < d1) {
            uint32_t i = co_rank(sA, na, sB, nb, d0);
            uint32_t j = d0 - i;
            for (uint32_t d = d0; d < d1; ++d) {
                uint32_t ea = i < na ? sA[i] : 0xffffffffu;
                uint32_t eb = j < nb ? sB[j] : 0xffffffffu;
                bool take_a = i < na && (j >= nb || (ea >> 2) <= (eb >> 2));
                if (take_a) {
                    if (j < nb && (ea >> 2) == (eb >> 2)) on_common<G>(ea >> 2, ea & 3u, eb & 3u, u, v, f, T, h);
                    ++i;
                } else {
                    ++j;
                }
            }
        }
        const uint32_t xt = co_rank(sA, na, sB, nb, total);
        __syncthreads();
        a_pos += xt;
        b_pos += total - xt;
    }
}

// ---------------------------------------------------------------- wave ----
constexpr int kWaveB = 64;
constexpr int kWaveTile = 1024;

__global__ __launch_bounds__(kWaveB) void k_census_wave(census_args L, unsigned int* next) {
    extern __shared__ unsigned long long lds[];
    __shared__ uint8_t T[64];
    __shared__ uint32_t sA[kWaveTile], sB[kWaveTile];
    unsigned long long* bins = lds;
    T[threadIdx.x] = c_table[threadIdx.x];
    hist_clear<kWaveB>(bins);
    __syncthreads();
    lane_hist<kWaveB> h{bins, (int)threadIdx.x};
    for (;;) {
        uint32_t d = 0;
        if (threadIdx.x == 0) d = atomicAdd(next, 1u);
        d = __shfl(d, 0, 64);
        if (d >= L.count) break;
        dyad_rec r = load_rec(L.dyads + d);
        if (threadIdx.x == 0) dyad_base<kWaveB>(r, L.tpre, L.n, T, h);
        merge_path<kWaveB, kWaveTile>(r, L.nbr, sA, sB, T, h);
    }
    hist_flush<kWaveB>(bins, L.acc);
}

// --------------------------------------------------------------- group ----
constexpr int kGroupB = 256;
constexpr int kGroupTile = 2048;

__global__ __launch_bounds__(kGroupB) void k_census_group(census_args L, unsigned int* next) {
    extern __shared__ unsigned long long lds[];
    __shared__ uint8_t T[64];
    __shared__ uint32_t sA[kGroupTile], sB[kGroupTile];
    __shared__ uint32_t cur;
    unsigned long long* bins = lds;
    if (threadIdx.x < 64) T[threadIdx.x] = c_table[threadIdx.x];
    hist_clear<kGroupB>(bins);
    __syncthreads();
    lane_hist<kGroupB> h{bins, (int)threadIdx.x};
    for (;;) {
        if (threadIdx.x == 0) cur = atomicAdd(next, 1u);
        __syncthreads();
        uint32_t d = cur;
        __syncthreads();
        if (d >= L.count) break;
        dyad_rec r = load_rec(L.dyads + d);
        if (threadIdx.x == 0) dyad_base<kGroupB>(r, L.tpre, L.n, T, h);
        merge_path<kGroupB, kGroupTile>(r, L.nbr, sA, sB, T, h);
    }
    hist_flush<kGroupB>(bins, L.acc);
}

__global__ void k_zero_u32(unsigned int* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

}  // namespace

hipError_t census_upload_table() {
    return hipMemcpyToSymbol(HIP_SYMBOL(c_table), kTable.t, sizeof(kTable.t));
}

hipError_t census_launch(const device_graph& g, const census_slices& sl, unsigned long long* acc,
                         unsigned int* counters, const census_config& cfg, hipStream_t s, hipEvent_t* ev) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, acc, kNumClasses);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, counters, kBuckets);
    for (int b = 0; b < kBuckets; ++b) {
        uint64_t cnt = sl.end[b] > sl.begin[b] ? sl.end[b] - sl.begin[b] : 0;
        if (ev) (void)hipEventRecord(ev[2 * b], s);
        if (cnt > 0) {
            census_args L{g.dyads + sl.begin[b], (uint32_t)cnt, g.nbr, g.tpre, (uint64_t)g.n, acc};
            if (b == 0) {
                uint32_t grid = (uint32_t)std::min<uint64_t>((cnt + kLaneB - 1) / kLaneB, cfg.lane_blocks);
                size_t sh = sizeof(unsigned long long) * kNumClasses * kLaneB;
                hipLaunchKernelGGL(k_census_lane, dim3(grid), dim3(kLaneB), sh, s, L);
            } else if (b == 1) {
                uint32_t grid = (uint32_t)std::min<uint64_t>(cnt, cfg.wave_blocks);
                size_t sh = sizeof(unsigned long long) * kNumClasses * kWaveB;
                hipLaunchKernelGGL(k_census_wave, dim3(grid), dim3(kWaveB), sh, s, L, counters + 1);
            } else {
                uint32_t grid = (uint32_t)std::min<uint64_t>(cnt, cfg.group_blocks);
                size_t sh = sizeof(unsigned long long) * kNumClasses * kGroupB;
                hipLaunchKernelGGL(k_census_group, dim3(grid), dim3(kGroupB), sh, s, L, counters + 2);
            }
        }
        if (ev) (void)hipEventRecord(ev[2 * b + 1], s);
    }
    return hipGetLastError();
}

}  // namespace tc
