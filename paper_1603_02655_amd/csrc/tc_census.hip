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
// Four execution modes over the buckets (key |N(u)| + |N(v)| - 2, and the
// longer row for the hub bucket):
//   lane  : one lane per record, the two rows compared 8 entries at a time;
//   wave  : one 64-lane wavefront per record, merge path over LDS-staged tiles;
//   group : one 256-lane workgroup per record, merge path over larger tiles;
//   hub   : one workgroup per group of runs of records that share an
//           endpoint (anchor), whose rows are staged in an LDS hash table and
//           probed by the other rows.
// The same kernels run over the dyad records (Tri = false) or over the
// forward-list edge records (Tri = true), where a shared vertex closes a
// triangle that is credited to its three dyads (on_triangle) and the per-dyad
// terms come from a separate pass over the neighbour entries (k_census_totals).
// Counts accumulate in LDS bins (per lane, per wavefront, or per signature in
// the hub mode); each workgroup adds its 16 sums to the graph's accumulators
// with one 64-bit global atomic per class when it finishes.
//
// The class of every code comes from a 64-entry table staged in LDS.  The
// single-graph kernels take the table as an argument: the 16-class table, or
// for the labelled (64-class) census one of three pass tables that send the
// codes whose (u, v) part is f to bin (code >> 2) and every other code to the
// discard bin (index kNumClasses), which is never flushed.
#include "tc_census.h"

namespace tc {

namespace {

__constant__ uint8_t c_table[64];

constexpr int kBins = kNumClasses + 1;     // 16 classes and the discard bin (kNumClasses)

// ---- class histograms in LDS ------------------------------------------------
// lane_bins: one private row of bins per lane (no contention; used where every
// lane works on its own dyad).  wave_bins: one row per wavefront updated with
// LDS atomics (used where a group shares a dyad and only shared neighbours and
// one lane's per-dyad totals are added).
template <int B>
struct lane_bins {
    static constexpr int kWords = kBins * B;
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

// block_bins: one row shared by the workgroup (LDS atomics; used where updates
// are rare next to the work that produces them).
template <int B>
struct block_bins {
    static constexpr int kWords = kBins;
    unsigned long long* bins;
    __device__ inline void add(uint32_t cls, unsigned long long x) { atomicAdd(&bins[cls], x); }
    __device__ inline void clear() {
        for (int i = threadIdx.x; i < kWords; i += B) bins[i] = 0;
    }
    __device__ inline void flush(unsigned long long* acc) {
        __syncthreads();
        if (threadIdx.x < kNumClasses && bins[threadIdx.x] != 0) atomicAdd(&acc[threadIdx.x], bins[threadIdx.x]);
    }
};

template <int B>
struct wave_bins {
    static constexpr int kWords = kBins * (B / 64);
    unsigned long long* bins;
    __device__ inline void add(uint32_t cls, unsigned long long x) {
        atomicAdd(&bins[(threadIdx.x >> 6) * kBins + cls], x);
    }
    __device__ inline void clear() {
        for (int i = threadIdx.x; i < kWords; i += B) bins[i] = 0;
    }
    __device__ inline void flush(unsigned long long* acc) {
        __syncthreads();
        if (threadIdx.x < kNumClasses) {
            unsigned long long s = 0;
            for (int w = 0; w < B / 64; ++w) s += bins[w * kBins + threadIdx.x];
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
    h.add(T[f], (unsigned long long)(n - du - dv));
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
    h.add(T[f], 1ull);                                    // |S| is one smaller
    if (w > v) {                                          // counted with its full code
        h.add(T[f | (fa << 2) | (fb << 4)], 1ull);
        h.add(T[f | (fa << 2)], ~0ull);                   // not a u-only vertex
    }
    if (w > u) h.add(T[f | (fb << 4)], ~0ull);            // not a v-only vertex
}

__device__ inline uint32_t swap_dir(uint32_t f) { return ((f & 1u) << 1) | (f >> 1); }

// A triangle {u, v, w}, u < v, found once (from the forward lists of its two
// first vertices in degree order): w is a shared vertex of each of its three
// dyads.  f = f_uv relative to u, fa = f_uw relative to u, fb = f_vw relative
// to v.
template <class H>
__device__ inline void on_triangle(uint32_t w, uint32_t fa, uint32_t fb, uint32_t u, uint32_t v, uint32_t f,
                                   const uint8_t* T, H& h) {
    const uint32_t sa = swap_dir(fa), sb = swap_dir(fb), sf = swap_dir(f);
    on_common(w, fa, fb, u, v, f, T, h);                      // dyad (u, v), third vertex w
    if (u < w) on_common(v, f, sb, u, w, fa, T, h);           // dyad (u, w), third vertex v
    else on_common(v, sb, f, w, u, sa, T, h);                 // dyad (w, u)
    if (v < w) on_common(u, sf, sa, v, w, fb, T, h);          // dyad (v, w), third vertex u
    else on_common(u, sa, sf, w, v, sb, T, h);                // dyad (w, v)
}

// What a shared vertex of the two rows of a record means: for dyad records a
// shared neighbour of the dyad; for forward-list edge records a triangle.
template <bool Tri, class H>
__device__ inline void on_shared(uint32_t w, uint32_t fa, uint32_t fb, uint32_t u, uint32_t v, uint32_t f,
                                 const uint8_t* T, H& h) {
    if constexpr (Tri) on_triangle(w, fa, fb, u, v, f, T, h);
    else on_common(w, fa, fb, u, v, f, T, h);
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
// One lane per record: the two rows, read from global memory (L1/L2 resident
// for the short rows of this bucket), compared in chunks.
constexpr int kLaneB = 256;

// The two rows are compared kLaneChunk entries at a time: a chunk of each is
// loaded with independent loads and every pair of the two chunks compared in
// registers; then the chunk whose last vertex is smaller is replaced.  No pair
// is compared twice and no shared vertex is missed: the chunk left in place
// holds no vertex below the last one of the chunk that is replaced, and the
// next chunk of a row starts above its current one.
constexpr uint32_t kLaneChunk = 8;

__device__ inline void load_chunk(const uint32_t* __restrict__ nbr, uint32_t pos, uint32_t end, uint32_t pad,
                                  uint32_t (&c)[kLaneChunk]) {
#pragma unroll
    for (uint32_t k = 0; k < kLaneChunk; ++k) c[k] = pos + k < end ? nbr[pos + k] : pad;
}

template <bool Tri, class H>
__device__ inline void lane_dyad(const dyad_rec& r, const uint32_t* __restrict__ nbr, const uint64_t* __restrict__ tpre,
                                 uint64_t n, const uint8_t* T, H& h) {
    dyad_totals t{};
    if constexpr (!Tri) t = load_totals(r, tpre);
    const uint32_t u = r.u, v = r.vf >> 2, f = r.vf & 3u;
    // pads: never equal to an entry or to each other (entries are below 2^25)
    constexpr uint32_t kPadA = 0xffffffffu, kPadB = 0xfffffff0u;
    uint32_t i = r.bu, j = r.bv;
    uint32_t A[kLaneChunk], B[kLaneChunk];
    load_chunk(nbr, i, r.eu, kPadA, A);
    load_chunk(nbr, j, r.ev, kPadB, B);
    for (;;) {
#pragma unroll
        for (uint32_t p = 0; p < kLaneChunk; ++p)
#pragma unroll
            for (uint32_t q = 0; q < kLaneChunk; ++q)
                if ((A[p] ^ B[q]) < 4u) on_shared<Tri>(A[p] >> 2, A[p] & 3u, B[q] & 3u, u, v, f, T, h);
        const uint32_t la = min(kLaneChunk, r.eu - i), lb = min(kLaneChunk, r.ev - j);
        uint32_t lastA = A[0], lastB = B[0];
#pragma unroll
        for (uint32_t k = 1; k < kLaneChunk; ++k) {
            lastA = k < la ? A[k] : lastA;
            lastB = k < lb ? B[k] : lastB;
        }
        if (lastA <= (lastB | 3u)) {
            i += kLaneChunk;
            if (i >= r.eu) break;
            load_chunk(nbr, i, r.eu, kPadA, A);
        } else {
            j += kLaneChunk;
            if (j >= r.ev) break;
            load_chunk(nbr, j, r.ev, kPadB, B);
        }
    }
    if constexpr (!Tri) add_totals(r, t, n, T, h);
}

// Dyad records add their per-dyad terms on every record: per-lane bins (in
// dynamic LDS).  Forward-list edge records only add on a triangle, which is
// rare per record: per-wavefront bins, and far less LDS.
template <bool Tri>
__global__ __launch_bounds__(kLaneB) void k_census_lane(census_args L) {
    extern __shared__ unsigned long long lds[];
    __shared__ uint8_t T[64];
    __shared__ unsigned long long wbins[Tri ? wave_bins<kLaneB>::kWords : 1];
    if (threadIdx.x < 64) T[threadIdx.x] = L.table[threadIdx.x];
    if constexpr (Tri) {
        wave_bins<kLaneB> h{wbins};
        h.clear();
        __syncthreads();
        for (uint64_t d = (uint64_t)blockIdx.x * kLaneB + threadIdx.x; d < L.count;
             d += (uint64_t)gridDim.x * kLaneB)
            lane_dyad<Tri>(load_rec(L.dyads + d), L.nbr, L.tpre, L.n, T, h);
        h.flush(L.acc);
    } else {
        lane_bins<kLaneB> h{lds};
        h.clear();
        __syncthreads();
        for (uint64_t d = (uint64_t)blockIdx.x * kLaneB + threadIdx.x; d < L.count;
             d += (uint64_t)gridDim.x * kLaneB)
            lane_dyad<Tri>(load_rec(L.dyads + d), L.nbr, L.tpre, L.n, T, h);
        h.flush(L.acc);
    }
}

// The per-dyad terms that need no intersection, for every dyad at once (the
// forward-list path), one lane per neighbour entry: entry y of row x, with
// the prefix counts of the direction bits, gives the typed counts of the
// entries after y in row x.  When y > x these are the entries of N(u) above v
// for the dyad (u, v) = (x, y); when y < x they are the entries of N(v) above
// u for the dyad (y, x).  The dyadic base n - |N(u)| - |N(v)| is split the
// same way: n - |N(x)| from the first side, -|N(x)| from the second.  The
// entry arrays are read coalesced, and the row's bounds and prefix counts at
// its end come in one 16-byte record shared by the row's entries.
//
// totals_entries: entries base + k * B + threadIdx.x (k < kPer) below `end`,
// their loads issued before any is used.
template <uint32_t kPer, uint32_t B, class H>
__device__ inline void totals_entries(uint64_t base, uint64_t end, const uint32_t* __restrict__ nbr,
                                      const uint32_t* __restrict__ owner, const uint4* __restrict__ rinfo,
                                      const uint64_t* __restrict__ tpre, uint64_t n, const uint8_t* T, H& h) {
    uint32_t x[kPer], ent[kPer];
    uint64_t rb[kPer], re[kPer], pend[kPer], pnext[kPer];
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint64_t e = base + k * B + threadIdx.x;
        x[k] = e < end ? owner[e] : 0u;
        ent[k] = e < end ? nbr[e] : 0u;
        pnext[k] = e < end ? tpre[e + 1] : 0ull;
    }
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint4 ri = rinfo[x[k]];
        rb[k] = ri.x;
        re[k] = ri.y;
        pend[k] = (uint64_t)ri.z | ((uint64_t)ri.w << 32);
    }
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint64_t e = base + k * B + threadIdx.x;
        if (e >= end) continue;
        const uint32_t y = ent[k] >> 2, fxy = ent[k] & 3u;
        const uint64_t pc = pend[k] - pnext[k];                 // direction bits after e in row x
        const uint64_t tot = re[k] - e - 1, out = pc & 0xffffffffull, in = pc >> 32;
        const uint64_t mut = out + in - tot;
        const bool first = y > x[k];                            // x plays u, else v
        const uint32_t f = first ? fxy : swap_dir(fxy);
        const uint32_t sh = first ? 2u : 4u;
        h.add(T[f], (unsigned long long)((first ? n : 0ull) - (re[k] - rb[k])));
        h.add(T[f | (1u << sh)], out - mut);
        h.add(T[f | (2u << sh)], in - mut);
        h.add(T[f | (3u << sh)], mut);
    }
}

constexpr uint32_t kTotalsPer = 4;   // entries per thread and step
constexpr uint32_t kTotalsSlots = 8; // distinct bins the totals pass can reach (any table here has <= 8)

// Adds straight to a graph's 16 accumulators in global memory.
struct global_bins {
    unsigned long long* acc;
    __device__ inline void add(uint32_t cls, unsigned long long x) { atomicAdd(&acc[cls], x); }
};

// Per-lane bins over a few slots: the totals pass reaches only the bins of the
// codes f, f | t << 2 and f | t << 4 (f, t in 1..3), at most kTotalsSlots of
// them, so a lane keeps one 64-bit slot per reachable bin (16 KB of LDS for
// 256 lanes instead of 35 KB).  The codes are remapped to slots in a table.
struct slot_bins {
    unsigned long long* bins;   // kTotalsSlots x kLaneB
    __device__ inline void add(uint32_t slot, unsigned long long x) {
        atomicAdd(&bins[slot * kLaneB + threadIdx.x], x);
    }
};

// Fills TS (code -> slot) and bin_of_slot for the reachable codes of table T;
// returns the number of slots, or 0 when more than kTotalsSlots bins are
// reachable.  One thread.
__device__ inline uint32_t totals_slots(const uint8_t* T, uint8_t* TS, uint32_t* bin_of_slot) {
    uint32_t ns = 0;
    bool all = true;
    for (uint32_t c = 0; c < 64; ++c) TS[c] = 0xff;
    for (uint32_t f = 1; f < 4; ++f)
        for (uint32_t j = 0; j < 7; ++j) {
            const uint32_t c = j == 0 ? f : (j <= 3 ? f | (j << 2) : f | ((j - 3) << 4));
            uint32_t sl = 0;
            while (sl < ns && bin_of_slot[sl] != T[c]) ++sl;
            if (sl == ns && ns < kTotalsSlots) bin_of_slot[ns++] = T[c];
            TS[c] = sl < ns ? (uint8_t)sl : (uint8_t)0xff;
            all = all && sl < ns;
        }
    return all ? ns : 0u;
}

// Sums the per-lane slots over a kLaneB workgroup into h (wavefront w takes
// slots w, w + 4) and clears them.
template <class H>
__device__ inline void slots_flush(unsigned long long* sbins, const uint32_t* bin_of_slot, uint32_t nslots, H& h) {
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    for (uint32_t sl = threadIdx.x >> 6; sl < nslots; sl += kLaneB / 64) {
        unsigned long long v = 0;
        for (uint32_t i = lane; i < kLaneB; i += 64) v += sbins[sl * kLaneB + i];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0 && v != 0 && bin_of_slot[sl] < kNumClasses) h.add(bin_of_slot[sl], v);
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < kTotalsSlots * kLaneB; k += kLaneB) sbins[k] = 0;
}

// Over the neighbour entries [e0, e1).
__global__ __launch_bounds__(kLaneB) void k_census_totals(const uint32_t* __restrict__ nbr,
                                                          const uint32_t* __restrict__ owner,
                                                          const uint4* __restrict__ rinfo,
                                                          const uint64_t* __restrict__ tpre, uint64_t e0, uint64_t e1,
                                                          uint64_t n, const uint8_t* __restrict__ table,
                                                          unsigned long long* __restrict__ acc) {
    __shared__ unsigned long long sbins[kTotalsSlots * kLaneB];
    __shared__ unsigned long long wbins[wave_bins<kLaneB>::kWords];
    __shared__ uint8_t T[64], TS[64];
    __shared__ uint32_t bin_of_slot[kTotalsSlots], s_nslots;
    if (threadIdx.x < 64) T[threadIdx.x] = table[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) s_nslots = totals_slots(T, TS, bin_of_slot);
    for (uint32_t k = threadIdx.x; k < kTotalsSlots * kLaneB; k += kLaneB) sbins[k] = 0;
    wave_bins<kLaneB> hw{wbins};
    hw.clear();
    __syncthreads();
    const uint32_t nslots = s_nslots;
    if (nslots) {
        slot_bins hs{sbins};
        for (uint64_t base = e0 + (uint64_t)blockIdx.x * kLaneB * kTotalsPer; base < e1;
             base += (uint64_t)gridDim.x * kLaneB * kTotalsPer)
            totals_entries<kTotalsPer, kLaneB>(base, e1, nbr, owner, rinfo, tpre, n, TS, hs);
        global_bins g{acc};
        slots_flush(sbins, bin_of_slot, nslots, g);
    } else {
        for (uint64_t base = e0 + (uint64_t)blockIdx.x * kLaneB * kTotalsPer; base < e1;
             base += (uint64_t)gridDim.x * kLaneB * kTotalsPer)
            totals_entries<kTotalsPer, kLaneB>(base, e1, nbr, owner, rinfo, tpre, n, T, hw);
        hw.flush(acc);
    }
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

template <int G, int TW, class Sync, bool Tri, class H>
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
                    if ((a ^ b) < 4u) on_shared<Tri>(a >> 2, a & 3u, b & 3u, u, v, f, T, h);
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
constexpr uint32_t kWaveChunk = 16;

// TW: entries of each row staged per round (the tunable LDS tile).
template <bool Tri, int TW>
__global__ __launch_bounds__(kWaveB) void k_census_wave(census_args L, unsigned int* ctr) {
    __shared__ unsigned long long bins[wave_bins<kWaveB>::kWords];
    __shared__ uint8_t T[64];
    __shared__ uint32_t sA[TW + 1], sB[TW + 1];
    __shared__ uint32_t s_xt;
    T[threadIdx.x] = L.table[threadIdx.x];
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
            if (!Tri && threadIdx.x == 0) t = load_totals(r, L.tpre);
            merge_path<kWaveB, TW, block_sync, Tri>(r, L.nbr, sA, sB, &s_xt, threadIdx.x, T, h);
            if (!Tri && threadIdx.x == 0) add_totals(r, t, L.n, T, h);
        }
        c = __shfl(cn, 0, 64);
    }
    h.flush(L.acc);
}

// --------------------------------------------------------------- group ----
constexpr uint32_t kGroupChunk = 2;

// B: workgroup size; TW: entries of each row staged per round (both tunable).
template <bool Tri, int B, int TW>
__global__ __launch_bounds__(B) void k_census_group(census_args L, unsigned int* ctr) {
    __shared__ unsigned long long bins[wave_bins<B>::kWords];
    __shared__ uint8_t T[64];
    __shared__ uint32_t sA[TW + 1], sB[TW + 1];
    __shared__ uint32_t s_xt, s_next;
    if (threadIdx.x < 64) T[threadIdx.x] = L.table[threadIdx.x];
    wave_bins<B> h{bins};
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
            if (!Tri && threadIdx.x == 0) t = load_totals(r, L.tpre);
            merge_path<B, TW, block_sync, Tri>(r, L.nbr, sA, sB, &s_xt, threadIdx.x, T, h);
            if (!Tri && threadIdx.x == 0) add_totals(r, t, L.n, T, h);
        }
        __syncthreads();
        c = s_next;
        __syncthreads();
    }
    h.flush(L.acc);
}


// ----------------------------------------------------------------- hub ----
// Hub records, grouped by anchor (their endpoint with the longer row) into
// hub tasks of up to kHubChunk records that share the anchor.  A workgroup
// takes kHubGroupTasks consecutive tasks at a time, stages the anchor rows into
// an LDS hash table (kHubTile entries in 4-slot buckets, the next bucket on
// overflow) -- the rows of several tasks together when they fit one tile, a
// longer row tile by tile -- and streams the other endpoint's row of every
// record against it: each entry of that row is probed once, in the tile whose
// vertex range holds it.  The anchor row is thus read once per task instead of
// once per record, and the work per record is proportional to the shorter row.
constexpr int kHubB = 256;
constexpr uint32_t kEmpty = 0xffffffffu;                 // never an entry (w < 2^23)
constexpr uint32_t kHubGather = 8;
constexpr uint32_t kHubFlushAfter = (1u << 24) - 1u;      // kHubB times this stays below 2^32

// First position in [lo, hi) of a sorted row whose vertex is >= w.
__device__ inline uint32_t find_first_ge(const uint32_t* __restrict__ nbr, uint32_t lo, uint32_t hi, uint32_t w) {
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if ((nbr[mid] >> 2) < w) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Geometry of one LDS tile of TILE anchor entries (the tunable hub tile): a
// hash table of TILE / 2 buckets of 4 slots (mean load 2 entries) and a filter
// of 8 bits per staged entry.  The table hashes a key (m << 23) | w (m the
// task's place in its group, w the vertex) folded to 24 bits, w + (m << 20),
// with a 24 x 24-bit multiply and keeps the top bits of the low 32 bits of the
// product (a full 32-bit multiply issues at a quarter of the rate).  The
// filter position of (m, w) is w * C + mix(m) (one multiply-add, mix(m)
// computed once per record): its top bits pick the filter word and its low
// five bits the bit, which is the shift count a 32-bit shift takes as it is.
// Only the placement depends on the hashes: a probe compares whole keys.
constexpr uint32_t kHubBucketMul = 0x9E3779u;            // odd 24-bit multipliers
constexpr uint32_t kHubFilterMul = 0x85EBCBu;
constexpr uint32_t kHubMemberMul = 0x9E3779B1u;          // odd 32-bit multiplier of the member index
__device__ inline uint32_t hub_fold(uint32_t key) { return (key & ((1u << 23) - 1u)) + ((key >> 23) << 20); }
// Low 32 bits of the product of the low 24 bits of a and b, unsigned (HIP's
// __umul24 returns a signed int, whose right shifts would be arithmetic).
__device__ inline uint32_t mul24(uint32_t a, uint32_t b) { return (uint32_t)__umul24(a, b); }
__device__ inline uint32_t hub_member_mix(uint32_t m) { return m * kHubMemberMul; }
template <uint32_t TILE>
struct hub_geom {
    static constexpr uint32_t kBuckets = TILE / 2;
    static constexpr uint32_t kSlots = 4 * kBuckets;
    static constexpr int kBucketBits = __builtin_ctz(kBuckets);
    static constexpr int kFilterLog = __builtin_ctz(TILE) + 3;
    static constexpr uint32_t kFilterBits = 1u << kFilterLog;
    static constexpr uint32_t kWordShift = 32 - (kFilterLog - 5);   // position >> kWordShift: the filter word
    static_assert((TILE & (TILE - 1)) == 0 && TILE >= 256 && TILE <= 4096, "power-of-two tile");
    static_assert(kFilterBits / 32 >= (uint32_t)kHubB / 8, "filter words");
    // from a folded key
    __device__ static inline uint32_t bucket_of(uint32_t fold) { return mul24(fold, kHubBucketMul) >> (32 - kBucketBits); }
    // vertex w (< 2^23) of the member whose hub_member_mix is mix
    __device__ static inline uint32_t filter_pos(uint32_t w, uint32_t mix) { return mul24(w, kHubFilterMul) + mix; }
};

// Buckets fill their slots in order, so a bucket whose last slot is empty
// ends the probe sequence of every vertex that hashes to it or before it.
template <uint32_t TILE>
__device__ inline void hub_insert(uint32_t* hash, uint32_t e) {
    using G = hub_geom<TILE>;
    uint32_t b = G::bucket_of(hub_fold(e >> 2));
    for (;;) {
        for (uint32_t s = 0; s < 4; ++s)
            if (atomicCAS(&hash[4 * b + s], kEmpty, e) == kEmpty) return;
        b = (b + 1) & (G::kBuckets - 1);
    }
}

// The whole bucket is read at once and its four slots compared without
// branches; the next bucket is read only when this one is full and holds no
// match.  key4 is the stored word with its direction bits cleared,
// (m << 25) | (w << 2), and fold the folded key.  A slot XOR key4 is below 4
// exactly when the slot holds the key (a key is stored at most once), and is
// then the slot's direction bits: the smallest of the four, clamped to 4, is
// the hit's direction bits, or 4 for no hit.
template <uint32_t TILE>
__device__ inline uint32_t hub_probe(const uint32_t* hash, uint32_t key4, uint32_t fold) {
    using G = hub_geom<TILE>;
    const uint4* h4 = reinterpret_cast<const uint4*>(hash);
    uint32_t b = G::bucket_of(fold);
    for (;;) {
        const uint4 q = h4[b];
        const uint32_t r = min(min(min(q.x ^ key4, q.y ^ key4), q.z ^ key4), min(q.w ^ key4, 4u));
        if (r < 4u || q.w == kEmpty) return r;
        b = (b + 1) & (G::kBuckets - 1);
    }
}

// Exclusive scan of a[0..count) in place on a 256-thread block (count <=
// 4 * 256); a[count .. count + kScanPad) receive the total.  wsum holds 4 words
// of LDS.
constexpr uint32_t kScanPad = 8;
template <uint32_t CH>
__device__ inline void block_scan_u32(uint32_t* a, uint32_t count, uint32_t* wsum) {
    constexpr uint32_t kPer = CH / kHubB;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
    uint32_t loc[kPer], s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t i = tid * kPer + k;
        loc[k] = s;
        s += i < count ? a[i] : 0u;
    }
    uint32_t incl = s;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(incl, o, 64);
        if ((int)lane >= o) incl += y;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (uint32_t w = 0; w < kHubB / 64; ++w) {
        base += w < wid ? wsum[w] : 0u;
        tot += wsum[w];
    }
    base += incl - s;
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t i = tid * kPer + k;
        if (i < count) a[i] = base + loc[k];
    }
    if (tid < kScanPad) a[count + tid] = tot;
    __syncthreads();
}

// What a shared vertex w of the dyad (or edge record) (u, v), u < v, adds to
// the census depends only on the direction bits f = f_uv, fa = f_uw, fb = f_vw
// (each 1, 2 or 3: the pairs are joined) and on where w lies: below u, between
// u and v, or above v (where = [w > u] + [w > v]).  The hub mode counts shared
// vertices per signature f | fa << 2 | fb << 4 | where << 6 (192 slots, 81 of
// them reachable) in one 32-bit LDS histogram per workgroup and turns the
// counts into class updates when it flushes.
constexpr uint32_t kSigs = 192;

// Scales every update of one signature by its count.
template <class H>
struct scaled_bins {
    H& h;
    unsigned long long c;
    __device__ inline void add(uint32_t cls, unsigned long long x) { h.add(cls, x * c); }
};

// Aligned blocks of kHubGather entries that hold the entries [p0, p1) of a row
// (row arrays are padded so that the last block is readable).
static_assert(kHubGather == 8, "a block is read as two 16-byte loads");
__device__ inline uint32_t hub_blocks(uint32_t p0, uint32_t p1) {
    return p1 > p0 ? (p1 + kHubGather - 1) / kHubGather - p0 / kHubGather : 0u;
}

// LDS of the hub mode: the hash table, one candidate ring per wavefront, four
// per-record arrays, scan scratch, the signature histogram, the filter and the
// task words.
constexpr uint32_t kHubRing = 128;   // candidates a wavefront holds between probe rounds
struct hub_lds {
    uint32_t* hash;   // hub_geom::kSlots, 16-byte aligned
    uint32_t* ring_e; // kHubRing x (kHubB / 64) candidates: the entry
    uint32_t* ring_m; // ... and the meta word of its record
    uint32_t* pos;    // next unprobed position in the other endpoint's row
    uint32_t* end;    // end of that row's entries in the current tile
    uint32_t* meta;   // (m << 26) | (x << 3) | (anchor is u) << 2 | f_uv, m the task's place in its group
    uint32_t* off;    // blocks of this tile, then their exclusive scan and kScanPad copies of the total
    uint32_t* wsum;   // 4 words
    uint32_t* sig;    // kSigs counts shared by the workgroup
    uint32_t* filt;   // hub_geom::kFilterBits bits: a vertex whose bit is clear is not in the tile
    uint32_t* tk;     // kHubTkWords: the tasks of the current chunk and their groups
};
// Words of hub_lds::tk: per task of the chunk its first record, record count,
// anchor-row start, anchor-row length and anchor; the group boundaries and
// their count; the record and row prefixes of the current group's members.
constexpr uint32_t kTkBegin = 0, kTkNrec = 8, kTkHb = 16, kTkLen = 24, kTkAnchor = 32, kTkGroups = 40,
                   kTkNGroups = 49, kTkRb = 50, kTkEb = 59, kHubTkWords = 68;
static_assert(kHubGroupTasks == 8, "the task words hold eight tasks");
// CH: the records of a group the LDS holds (kHubChunk, or half of it for
// graphs whose tasks and groups are half-size).
template <uint32_t TILE, uint32_t CH>
constexpr uint32_t hub_lds_words() {
    return hub_geom<TILE>::kSlots + 2 * kHubRing * (kHubB / 64) + 3 * CH + (CH + kScanPad) + 4 + kSigs +
           hub_geom<TILE>::kFilterBits / 32 + kHubTkWords;
}

// Wavefronts per SIMD the hub kernels are compiled for: seven (the best
// measured with 1024-entry tiles), or as many workgroups as the LDS of a CU
// (160 KiB) holds for larger tiles (the kernels' other LDS takes < 256 bytes).
template <uint32_t TILE, uint32_t CH>
constexpr uint32_t hub_waves_per_simd() {
    return (163840u / (4u * hub_lds_words<TILE, CH>() + 256u)) < 7u ? (163840u / (4u * hub_lds_words<TILE, CH>() + 256u))
                                                                   : 7u;
}

template <uint32_t TILE, uint32_t CH>
__device__ inline hub_lds hub_carve(uint32_t* base) {
    uint32_t* p = base;
    hub_lds S;
    S.hash = p;  p += hub_geom<TILE>::kSlots;
    S.ring_e = p;  p += kHubRing * (kHubB / 64);
    S.ring_m = p;  p += kHubRing * (kHubB / 64);
    S.pos = p;   p += CH;
    S.end = p;   p += CH;
    S.meta = p;  p += CH;
    S.off = p;   p += CH + kScanPad;
    S.wsum = p;  p += 4;
    S.sig = p;   p += kSigs;
    S.filt = p;  p += hub_geom<TILE>::kFilterBits / 32;
    S.tk = p;
    return S;
}

__device__ inline void hub_bins_clear(const hub_lds& S) {
    for (uint32_t k = threadIdx.x; k < kSigs; k += kHubB) S.sig[k] = 0;
}

// Adds the signature counts to h (one thread per signature) and clears them.
template <bool Tri, class H>
__device__ inline void hub_bins_flush(const hub_lds& S, const uint8_t* T, H& h) {
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < kSigs; k += kHubB) {
        const uint32_t c = S.sig[k];
        if (c == 0) continue;
        S.sig[k] = 0;
        const uint32_t f = k & 3u, fa = (k >> 2) & 3u, fb = (k >> 4) & 3u, where = k >> 6;
        if (f == 0 || fa == 0 || fb == 0) continue;   // never counted
        // ids that put w below u, between u and v, or above v
        const uint32_t u = 1u, v = 3u, w = where * 2u;
        scaled_bins<H> sh{h, (unsigned long long)c};
        on_shared<Tri>(w, fa, fb, u, v, f, T, sh);
    }
    __syncthreads();
}

// One group of hub tasks on the whole workgroup (kHubB threads): members
// [js, js + M) of the chunk's tasks, whose anchor rows together fit one tile
// unless the group is a single task.  Per tile of the members' concatenated
// anchor rows: clear and fill the hash table (an entry of member m is stored
// with m above its 25 bits, so each record matches its own anchor only);
// count, for every record, the aligned blocks of kHubGather entries that hold
// the entries of the other row in the tile's vertex range; scan the counts;
// then each wavefront walks a quarter of the flattened block list, one block
// per lane, and probes the entries that pass the tile's filter 64 at a time.
// A hit adds one to the workgroup's count of the hit's signature.
template <bool Tri, uint32_t TILE, uint32_t CH, class H>
__device__ inline void hub_group_run(uint32_t js, uint32_t M, const dyad_rec* __restrict__ dyads,
                                     const uint32_t* __restrict__ nbr, const uint64_t* __restrict__ tpre, uint64_t n,
                                     uint32_t u_lo, uint32_t u_hi, const hub_lds& S, const uint8_t* T, H& h,
                                     uint32_t& since) {
    using G = hub_geom<TILE>;
    const uint32_t tid = threadIdx.x;
    const uint32_t* rb = S.tk + kTkRb;   // record prefix of the members (M + 1 words)
    const uint32_t* eb = S.tk + kTkEb;   // anchor-row prefix of the members (M + 1 words)
    const uint32_t nrec = rb[M], total = eb[M];
    const bool multi_tile = total > TILE;   // a single task
    for (uint32_t i = tid; i < nrec; i += kHubB) {
        uint32_t m = 0;
        while (m + 1 < M && rb[m + 1] <= i) ++m;
        const uint32_t a = S.tk[kTkAnchor + js + m];
        const dyad_rec r = load_rec(dyads + S.tk[kTkBegin + js + m] + (i - rb[m]));
        const bool anchor_u = r.u == a;
        const uint32_t x = anchor_u ? (r.vf >> 2) : r.u;
        const uint32_t xb = anchor_u ? r.bv : r.bu, xe = anchor_u ? r.ev : r.eu;
        const bool in = r.u >= u_lo && r.u < u_hi;
        const uint32_t p0 = in ? xb : xe;   // outside the requested range: nothing to probe
        S.pos[i] = p0;
        S.meta[i] = (m << 26) | (x << 3) | (anchor_u ? 4u : 0u) | (r.vf & 3u);
        if (!multi_tile) {
            S.end[i] = xe;
            S.off[i] = hub_blocks(p0, xe);
        }
        if (!Tri && in) add_totals(r, load_totals(r, tpre), n, T, h);
    }
    for (uint32_t tb = 0; tb < total; tb += TILE) {
        const uint32_t te = min(total, tb + TILE);
        for (uint32_t k = tid; k < G::kSlots; k += kHubB) S.hash[k] = kEmpty;
        for (uint32_t k = tid; k < G::kFilterBits / 32; k += kHubB) S.filt[k] = 0;
        __syncthreads();
        for (uint32_t f = tb + tid; f < te; f += kHubB) {
            uint32_t m = 0;
            while (m + 1 < M && eb[m + 1] <= f) ++m;
            const uint32_t v = nbr[S.tk[kTkHb + js + m] + (f - eb[m])];
            hub_insert<TILE>(S.hash, (m << 25) | v);
            const uint32_t fp = G::filter_pos(v >> 2, hub_member_mix(m));
            atomicOr(&S.filt[fp >> G::kWordShift], 1u << (fp & 31u));
        }
        if (multi_tile) {
            const uint32_t hb = S.tk[kTkHb + js], a = S.tk[kTkAnchor + js];
            const uint32_t w_end = te < total ? (nbr[hb + te] >> 2) : kEmpty;
            for (uint32_t i = tid; i < nrec; i += kHubB) {
                const uint32_t p0 = S.pos[i];
                uint32_t xe = p0;
                if (p0 != 0xffffffffu) {
                    const dyad_rec r = load_rec(dyads + S.tk[kTkBegin + js] + i);
                    xe = r.u == a ? r.ev : r.eu;
                }
                const uint32_t p1 = w_end == kEmpty ? xe : find_first_ge(nbr, p0, xe, w_end);
                S.end[i] = p1;
                S.off[i] = hub_blocks(p0, p1);
            }
        }
        __syncthreads();
        block_scan_u32<CH>(S.off, nrec, S.wsum);
        const uint32_t P = S.off[nrec];
        // The shared 32-bit signature counts grow by at most kHubGather * P in
        // this tile: they are flushed first when the tiles since the last flush
        // could take them past 2^32 (`per` is the same on every thread).
        const uint32_t per = (uint32_t)min((uint64_t)kHubGather * P / kHubB + 1, (uint64_t)kHubFlushAfter);
        if (since + per > kHubFlushAfter) {
            hub_bins_flush<Tri>(S, T, h);
            since = 0;
        }
        since += per;
        // The rows to probe are cut into aligned blocks of kHubGather entries
        // (a row's first and last block masked to the row).  Wavefront w takes
        // the w-th quarter [q0, q1) of the flattened list of blocks and walks it
        // 64 blocks at a time, one block per lane, read with two 16-byte loads.
        // A lane finds the record of its next block from the four record
        // starts after its current one (by bisection beyond).  Entries that
        // pass the filter are appended to the wavefront's ring of candidates,
        // and every 64 candidates are probed together, one per lane.
        const uint32_t lane = tid & 63u, wid = tid >> 6;
        constexpr uint32_t kWaves = kHubB / 64;
        const uint32_t q0 = (uint32_t)(((uint64_t)P * wid) / kWaves), q1 = (uint32_t)(((uint64_t)P * (wid + 1)) / kWaves);
        uint32_t* ring_e = S.ring_e + wid * kHubRing;
        uint32_t* ring_m = S.ring_m + wid * kHubRing;
        uint32_t cnt = 0;   // the same on every lane: ring[0, cnt) waits to be probed
        // Probes ring[l] on the lanes l < c (c <= 64): a hit adds one to the
        // count of its signature.  The hit's direction bits fh are relative
        // to the anchor a, the candidate's fx to the other endpoint x; the
        // anchor is u (then fa = fh, fb = fx) or v (fa = fx, fb = fh).
        auto probe_round = [&](uint32_t c) {
            wave_sync{}();
            if (lane < c) {
                const uint32_t qe = ring_e[lane], qm = ring_m[lane];
                const uint32_t w = qe >> 2, mm = qm >> 26;
                const uint32_t fh = hub_probe<TILE>(S.hash, (qe & ~3u) | (mm << 25), w + (mm << 20));
                if (fh < 4u) {
                    const uint32_t a = S.tk[kTkAnchor + js + mm];
                    const uint32_t x = (qm >> 3) & ((1u << 23) - 1u);
                    const uint32_t sx = (qm & 4u) ? 4u : 2u;
                    const uint32_t code = (qm & 3u) | ((qe & 3u) << sx) | (fh << (6u - sx));
                    const uint32_t where = (w > a ? 1u : 0u) + (w > x ? 1u : 0u);
                    atomicAdd(&S.sig[code | (where << 6)], 1u);
                }
            }
            wave_sync{}();
        };
        if (q0 < q1) {
            uint32_t i = 0;
            {
                // lanes past the quarter's end take its last record and gather nothing
                const uint32_t first = min(q0 + lane, q1 - 1u);
                uint32_t hi = nrec;                     // record holding `first`: off[i] <= first < off[i+1]
                while (hi - i > 1) {
                    const uint32_t mid = (i + hi) >> 1;
                    if (S.off[mid] <= first) i = mid; else hi = mid;
                }
            }
            uint32_t next = S.off[i + 1], p0 = S.pos[i], p1 = S.end[i], m = S.meta[i];
            uint32_t mix = hub_member_mix(m >> 26);
            uint32_t bb = p0 / kHubGather - S.off[i];   // block of flattened index f: bb + f (mod 2^32)
            for (uint32_t win = q0; win < q1; win += 64u) {
                // lanes past the quarter's end read its last block and keep no entry of it
                const uint32_t f = min(win + lane, q1 - 1u);
                if (f >= next) {
                    // The record of f from the next four record starts
                    // (off[nrec ..] = P > f past the last record), and by
                    // bisection when it lies further ahead.
                    const uint32_t o2 = S.off[i + 2], o3 = S.off[i + 3], o4 = S.off[i + 4], o5 = S.off[i + 5];
                    i += 1u + (f >= o2 ? 1u : 0u) + (f >= o3 ? 1u : 0u) + (f >= o4 ? 1u : 0u) + (f >= o5 ? 1u : 0u);
                    next = S.off[i + 1];
                    if (f >= next) {
                        uint32_t hi = nrec;
                        while (hi - i > 1) {
                            const uint32_t mid = (i + hi) >> 1;
                            if (S.off[mid] <= f) i = mid; else hi = mid;
                        }
                        next = S.off[i + 1];
                    }
                    p0 = S.pos[i];
                    p1 = S.end[i];
                    m = S.meta[i];
                    mix = hub_member_mix(m >> 26);
                    bb = p0 / kHubGather - S.off[i];
                }
                const uint32_t b0 = (bb + f) * kHubGather;   // first entry of the block: b0 < p1, p0 < b0 + 8
                const uint4* src = reinterpret_cast<const uint4*>(nbr + b0);
                const uint4 lo4 = src[0], hi4 = src[1];
                const uint32_t e[kHubGather] = {lo4.x, lo4.y, lo4.z, lo4.w, hi4.x, hi4.y, hi4.z, hi4.w};
                const uint32_t klo = p0 > b0 ? p0 - b0 : 0u, khi = min(p1 - b0, kHubGather);
                // bit k: word k is an entry of the row (none past the quarter's end)
                const uint32_t vm = win + lane < q1 ? ((1u << khi) - 1u) & ~((1u << klo) - 1u) : 0u;
                // Filter: the word of every entry first, then the bits.
                uint32_t fp[kHubGather], fw[kHubGather];
#pragma unroll
                for (uint32_t k = 0; k < kHubGather; ++k) {
                    fp[k] = G::filter_pos(e[k] >> 2, mix);
                    fw[k] = S.filt[fp[k] >> G::kWordShift];
                }
                // appends: the entries that pass go to ring[cnt ..] in lane order
#pragma unroll
                for (uint32_t k = 0; k < kHubGather; ++k) {
                    const bool pass = ((fw[k] >> (fp[k] & 31u)) & (vm >> k) & 1u) != 0u;
                    const unsigned long long bal = __builtin_amdgcn_ballot_w64(pass);
                    // (the lanes of the mask: the same lanes as pass, without a second compare)
                    if (__builtin_amdgcn_inverse_ballot_w64(bal)) {
                        const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)bal, cnt));
                        ring_e[r] = e[k];
                        ring_m[r] = m;
                    }
                    cnt += (uint32_t)__popcll(bal);
                    if (cnt >= 64u) {
                        probe_round(64u);
                        cnt -= 64u;
                        // the rest moves to the front
                        uint32_t te = 0, tm = 0;
                        if (lane < cnt) {
                            te = ring_e[64u + lane];
                            tm = ring_m[64u + lane];
                        }
                        wave_sync{}();
                        if (lane < cnt) {
                            ring_e[lane] = te;
                            ring_m[lane] = tm;
                        }
                    }
                }
            }
            if (cnt != 0) probe_round(cnt);
        }
        __syncthreads();
        if (multi_tile)
            for (uint32_t i = tid; i < nrec; i += kHubB) S.pos[i] = S.end[i];
        __syncthreads();
    }
}

// Hub tasks [t0, t1) (at most kHubGroupTasks) on the whole workgroup: their
// descriptors and anchor rows are read once, and runs of consecutive tasks
// whose records fit one chunk (`chunk` <= CH records, the graph's) and
// whose anchor rows fit one tile are processed together; a task whose anchor
// row spans several tiles runs alone.
template <bool Tri, uint32_t TILE, uint32_t CH, class H>
__device__ inline void hub_chunk_run(const hub_task* __restrict__ tasks, uint32_t t0, uint32_t t1,
                                     const dyad_rec* __restrict__ dyads, const uint32_t* __restrict__ nbr,
                                     const uint64_t* __restrict__ tpre, uint64_t n, uint32_t u_lo, uint32_t u_hi,
                                     uint32_t chunk, const hub_lds& S, const uint8_t* T, H& h, uint32_t& since) {
    const uint32_t tid = threadIdx.x, nt = t1 - t0;
    if (tid < nt) {
        const hub_task tk = tasks[t0 + tid];
        const dyad_rec r0 = load_rec(dyads + tk.begin);
        const bool au = r0.u == tk.anchor;
        const uint32_t hb = au ? r0.bu : r0.bv, he = au ? r0.eu : r0.ev;
        S.tk[kTkBegin + tid] = tk.begin;
        S.tk[kTkNrec + tid] = tk.end - tk.begin;
        S.tk[kTkHb + tid] = hb;
        S.tk[kTkLen + tid] = he - hb;
        S.tk[kTkAnchor + tid] = tk.anchor;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t ng = 0, sr = 0, se = 0;
        S.tk[kTkGroups] = 0;
        for (uint32_t j = 0; j < nt; ++j) {
            const uint32_t r = S.tk[kTkNrec + j], l = S.tk[kTkLen + j];
            if (j > S.tk[kTkGroups + ng] && (l > TILE || sr + r > chunk || se + l > TILE)) {
                S.tk[kTkGroups + ++ng] = j;
                sr = 0;
                se = 0;
            }
            sr += r;
            se += l;
        }
        S.tk[kTkGroups + ++ng] = nt;
        S.tk[kTkNGroups] = ng;
    }
    __syncthreads();
    const uint32_t ng = S.tk[kTkNGroups];
    for (uint32_t g = 0; g < ng; ++g) {
        const uint32_t js = S.tk[kTkGroups + g], M = S.tk[kTkGroups + g + 1] - js;
        if (tid == 0) {
            uint32_t r = 0, e = 0;
            for (uint32_t m = 0; m < M; ++m) {
                S.tk[kTkRb + m] = r;
                S.tk[kTkEb + m] = e;
                r += S.tk[kTkNrec + js + m];
                e += S.tk[kTkLen + js + m];
            }
            S.tk[kTkRb + M] = r;
            S.tk[kTkEb + M] = e;
        }
        __syncthreads();
        hub_group_run<Tri, TILE, CH>(js, M, dyads, nbr, tpre, n, u_lo, u_hi, S, T, h, since);
        __syncthreads();
    }
}

template <bool Tri, uint32_t TILE, uint32_t CH>
__global__ __launch_bounds__(kHubB)
__attribute__((amdgpu_waves_per_eu(hub_waves_per_simd<TILE, CH>(), hub_waves_per_simd<TILE, CH>()))) void k_census_hub(
    census_args L, const hub_task* __restrict__ tasks, uint32_t ntasks, uint32_t ngroups, uint32_t g0, uint32_t g1,
    unsigned int* ctr) {
    __shared__ __attribute__((aligned(16))) uint32_t hub_words[hub_lds_words<TILE, CH>()];
    __shared__ unsigned long long bins[block_bins<kHubB>::kWords];
    __shared__ uint8_t T[64];
    __shared__ uint32_t s_next;
    if (threadIdx.x < 64) T[threadIdx.x] = L.table[threadIdx.x];
    block_bins<kHubB> h{bins};
    h.clear();
    const hub_lds S = hub_carve<TILE, CH>(hub_words);
    hub_bins_clear(S);
    __syncthreads();
    uint32_t since = 0;
    const uint32_t xcd = blockIdx.x % kXcds;
    // task groups g0 + k, k taken from the counters, below g1 (<= ngroups)
    if (threadIdx.x == 0) s_next = g0 + take_chunk(ctr, xcd);
    __syncthreads();
    uint32_t c = s_next;
    __syncthreads();
    while (c < g1) {
        if (threadIdx.x == 0) s_next = g0 + take_chunk(ctr, xcd);
        const uint32_t t0 = tasks[c].group, t1 = c + 1 < ngroups ? tasks[c + 1].group : ntasks;
        hub_chunk_run<Tri, TILE, CH>(tasks, t0, t1, L.dyads, L.nbr, L.tpre, L.n, L.u_lo, L.u_hi, L.hub_chunk, S, T, h,
                                 since);
        c = s_next;
        __syncthreads();
    }
    hub_bins_flush<Tri>(S, T, h);
    h.flush(L.acc);
}

// --------------------------------------------------------------- batch ----
// Two persistent launches over the work items of many resident graphs: the
// hub task groups of every graph (k_census_batch_hub, seven wavefronts per SIMD
// like the single-graph hub kernel), then the other items (k_census_batch).  A
// workgroup takes items one at a time (per-XCD counters); an item is a slice
// of one graph's bucket, over its dyad records or its forward-list edge
// records: up to 256 lane-mode records (one per thread), up to
// 4 * kBatchWavePerItem wave-mode records (wavefront w takes every fourth), one
// group-mode record, one group of hub tasks, or a chunk of the totals pass.  Counts go
// to per-wavefront bins that are flushed into the graph's 16 accumulators
// whenever the workgroup moves to another graph.
constexpr int kBatchB = 256;
// The tile area of k_census_batch for wave-mode tile TW (the tunable batch
// tile; the group-mode tile is 4 TW): four wavefronts' pairs of TW-entry
// tiles, or one pair of 4 TW-entry tiles.
template <int TW>
constexpr int batch_tile_words() {
    return (4 * 2 * (TW + 1) > 2 * (4 * TW + 1)) ? 4 * 2 * (TW + 1) : 2 * (4 * TW + 1);
}
static_assert(kBatchTotalsPerItem % kBatchB == 0, "totals items are whole steps of the workgroup");
static_assert(kBatchB == kLaneB, "the slot helpers assume 256-lane workgroups");

template <bool Tri, int TW, class H>
__device__ inline void batch_item(uint32_t kind, const work_item& it, const graph_desc& g, uint32_t* tiles,
                                  uint32_t* s_xt, const uint8_t* T, H& h) {
    const uint32_t tid = threadIdx.x, wid = tid >> 6, lane = tid & 63u;
    const dyad_rec* recs = Tri ? g.edges : g.dyads;
    const uint32_t* nbr = Tri ? g.fwd : g.nbr;
    if (kind == kItemLane) {
        const uint32_t d = it.begin + tid;
        if (d < it.end) lane_dyad<Tri>(load_rec(recs + d), nbr, g.tpre, g.n, T, h);
    } else if (kind == kItemWave) {
        uint32_t* sA = tiles + wid * 2 * (TW + 1);
        uint32_t* sB = sA + TW + 1;
        for (uint32_t d = it.begin + wid; d < it.end; d += kBatchB / 64) {
            const dyad_rec r = load_rec(recs + d);
            dyad_totals t{};
            if (!Tri && lane == 0) t = load_totals(r, g.tpre);
            merge_path<64, TW, wave_sync, Tri>(r, nbr, sA, sB, &s_xt[wid], lane, T, h);
            if (!Tri && lane == 0) add_totals(r, t, g.n, T, h);
        }
    } else if (kind == kItemGroup) {
        const dyad_rec r = load_rec(recs + it.begin);
        dyad_totals t{};
        if (!Tri && tid == 0) t = load_totals(r, g.tpre);
        merge_path<kBatchB, 4 * TW, block_sync, Tri>(r, nbr, tiles, tiles + 4 * TW + 1, &s_xt[0], tid, T, h);
        if (!Tri && tid == 0) add_totals(r, t, g.n, T, h);
    }
}

template <uint32_t TILE, uint32_t CH>
__global__ __launch_bounds__(kHubB)
__attribute__((amdgpu_waves_per_eu(hub_waves_per_simd<TILE, CH>(), hub_waves_per_simd<TILE, CH>()))) void
k_census_batch_hub(
    const graph_desc* __restrict__ G, const work_item* __restrict__ items, const uint32_t* __restrict__ nums,
    unsigned long long* __restrict__ accs, unsigned int* __restrict__ ctr) {
    __shared__ __attribute__((aligned(16))) uint32_t hub_words[hub_lds_words<TILE, CH>()];
    __shared__ unsigned long long bins[block_bins<kHubB>::kWords];
    __shared__ uint8_t T[64];
    __shared__ uint32_t s_next;
    if (threadIdx.x < 64) T[threadIdx.x] = c_table[threadIdx.x];
    block_bins<kHubB> h{bins};
    h.clear();
    const hub_lds S = hub_carve<TILE, CH>(hub_words);
    hub_bins_clear(S);
    __syncthreads();
    const uint32_t count = nums[0];
    const uint32_t xcd = blockIdx.x % kXcds;
    uint32_t cur = 0xffffffffu, since = 0;
    bool cur_tri = false;
    if (threadIdx.x == 0) s_next = take_chunk(ctr, xcd);
    __syncthreads();
    uint32_t idx = s_next;
    __syncthreads();
    while (idx < count) {
        if (threadIdx.x == 0) s_next = take_chunk(ctr, xcd);
        const work_item it = items[idx];
        if (it.graph != cur) {
            if (cur != 0xffffffffu) {
                if (cur_tri) hub_bins_flush<true>(S, T, h);
                else hub_bins_flush<false>(S, T, h);
                h.flush(accs + (uint64_t)kNumClasses * cur);
                __syncthreads();
                h.clear();
            }
            cur = it.graph;
            cur_tri = (it.kind & kItemTri) != 0;   // one path per graph
            since = 0;
            __syncthreads();
        }
        const graph_desc g = G[it.graph];
        for (uint32_t k = it.begin; k < it.end; ++k) {
            if (cur_tri) {
                const uint32_t t0 = g.edge_tasks[k].group;
                const uint32_t t1 = k + 1 < g.tri_groups ? g.edge_tasks[k + 1].group : g.tri_tasks;
                hub_chunk_run<true, TILE, CH>(g.edge_tasks, t0, t1, g.edges, g.fwd, g.tpre, g.n, 0u, 0xffffffffu,
                                          g.tri_chunk, S, T, h,
                                          since);
            } else {
                const uint32_t t0 = g.hub_tasks[k].group;
                const uint32_t t1 = k + 1 < g.hub_groups ? g.hub_tasks[k + 1].group : g.hub_ntasks;
                hub_chunk_run<false, TILE, CH>(g.hub_tasks, t0, t1, g.dyads, g.nbr, g.tpre, g.n, 0u, 0xffffffffu,
                                           g.hub_chunk, S, T, h,
                                           since);
            }
        }
        idx = s_next;
        __syncthreads();
    }
    if (cur != 0xffffffffu) {
        if (cur_tri) hub_bins_flush<true>(S, T, h);
        else hub_bins_flush<false>(S, T, h);
        h.flush(accs + (uint64_t)kNumClasses * cur);
    }
}

// Compiled for seven wavefronts per SIMD with 512-entry tiles (72 VGPRs; the
// few values that no longer fit are reloaded once per item): the kernel waits
// on memory, and more resident waves hide more of it than the spills cost.
// Larger tiles are held to fewer waves by their LDS and keep their registers.
template <int TW>
constexpr int batch_min_waves() { return TW <= 512 ? 7 : 1; }
template <int TW>
__global__ __launch_bounds__(kBatchB) __attribute__((amdgpu_waves_per_eu(batch_min_waves<TW>()))) void k_census_batch(
    const graph_desc* __restrict__ G, const work_item* __restrict__ items, const uint32_t* __restrict__ num_items,
    unsigned long long* __restrict__ accs, unsigned int* __restrict__ ctr) {
    static_assert(2 * kTotalsSlots * kBatchB <= batch_tile_words<TW>(), "per-lane slots fit in the tile area");
    __shared__ __attribute__((aligned(16))) uint32_t tiles[batch_tile_words<TW>()];
    __shared__ unsigned long long bins[wave_bins<kBatchB>::kWords];
    __shared__ uint8_t T[64], TS[64];
    __shared__ uint32_t s_xt[kBatchB / 64], s_next, bin_of_slot[kTotalsSlots], s_nslots;
    if (threadIdx.x < 64) T[threadIdx.x] = c_table[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) s_nslots = totals_slots(T, TS, bin_of_slot);
    wave_bins<kBatchB> h{bins};
    h.clear();
    const uint32_t first = num_items[0], count = num_items[1];
    const uint32_t xcd = blockIdx.x % kXcds;
    const uint32_t tid = threadIdx.x;
    uint32_t cur = 0xffffffffu;
    if (tid == 0) s_next = first + take_chunk(ctr, xcd);
    __syncthreads();
    uint32_t idx = s_next;
    __syncthreads();
    while (idx < count) {
        if (tid == 0) s_next = first + take_chunk(ctr, xcd);
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
        if (it.kind == kItemTotals) {
            // per-lane slots in the (idle) tile area, summed into the
            // wavefront bins at the end of the item
            const uint32_t nslots = s_nslots;
            if (nslots) {
                unsigned long long* sbins = reinterpret_cast<unsigned long long*>(tiles);
                for (uint32_t k = tid; k < kTotalsSlots * kBatchB; k += kBatchB) sbins[k] = 0;
                __syncthreads();
                slot_bins hs{sbins};
                for (uint32_t b0 = it.begin; b0 < it.end; b0 += kTotalsPer * kBatchB)
                    totals_entries<kTotalsPer, kBatchB>(b0, it.end, g.nbr, g.owner, g.rinfo, g.tpre, g.n, TS,
                                                        hs);
                slots_flush(sbins, bin_of_slot, nslots, h);
            } else {
                for (uint32_t b0 = it.begin; b0 < it.end; b0 += kTotalsPer * kBatchB)
                    totals_entries<kTotalsPer, kBatchB>(b0, it.end, g.nbr, g.owner, g.rinfo, g.tpre, g.n, T, h);
            }
        }
        else if (it.kind & kItemTri)
            batch_item<true, TW>(it.kind & 3u, it, g, tiles, s_xt, T, h);
        else
            batch_item<false, TW>(it.kind, it, g, tiles, s_xt, T, h);
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

bool tile_supported(uint32_t hub_tile, uint32_t wave_tile, uint32_t group_tile, uint32_t group_size,
                    uint32_t batch_tile) {
    const bool hub = hub_tile == 512 || hub_tile == 1024 || hub_tile == 2048;
    const bool wave = wave_tile == 512 || wave_tile == 1024 || wave_tile == 2048;
    const bool group = group_tile == 2048 || group_tile == 4096 || group_tile == 8192;
    const bool gsize = group_size == 256 || group_size == 512;
    const bool batch = batch_tile == 512 || batch_tile == 1024 || batch_tile == 2048;
    return hub && wave && group && gsize && batch;
}

namespace {

template <uint32_t HT, int BT>
void launch_batch_kernels(const graph_desc* descs, const work_item* items, const uint32_t* nums,
                          unsigned long long* accs, unsigned int* counters, uint32_t grid, uint32_t hub_grid,
                          uint32_t hub_chunk, hipStream_t s) {
    if (hub_chunk <= kHubChunk / 2)
        hipLaunchKernelGGL((k_census_batch_hub<HT, kHubChunk / 2>), dim3(hub_grid), dim3(kHubB), 0, s, descs, items,
                           nums, accs, counters);
    else
        hipLaunchKernelGGL((k_census_batch_hub<HT, kHubChunk>), dim3(hub_grid), dim3(kHubB), 0, s, descs, items, nums,
                           accs, counters);
    hipLaunchKernelGGL(k_census_batch<BT>, dim3(grid), dim3(kBatchB), 0, s, descs, items, nums, accs,
                       counters + kXcds);
}

template <uint32_t HT>
void launch_batch_bt(uint32_t bt, const graph_desc* descs, const work_item* items, const uint32_t* nums,
                     unsigned long long* accs, unsigned int* counters, uint32_t grid, uint32_t hub_grid,
                     uint32_t hub_chunk, hipStream_t s) {
    if (bt == 512) launch_batch_kernels<HT, 512>(descs, items, nums, accs, counters, grid, hub_grid, hub_chunk, s);
    else if (bt == 1024)
        launch_batch_kernels<HT, 1024>(descs, items, nums, accs, counters, grid, hub_grid, hub_chunk, s);
    else launch_batch_kernels<HT, 2048>(descs, items, nums, accs, counters, grid, hub_grid, hub_chunk, s);
}

}  // namespace

hipError_t batch_launch(const graph_desc* descs, const work_item* items, const uint32_t* nums,
                        unsigned long long* accs, uint64_t acc_words, unsigned int* counters, uint32_t grid,
                        uint32_t hub_grid, uint32_t hub_tile, uint32_t batch_tile, uint32_t hub_chunk, hipStream_t s) {
    if (!tile_supported(hub_tile, 1024, 4096, 256, batch_tile)) return hipErrorInvalidValue;
    uint32_t zb = (uint32_t)std::min<uint64_t>((acc_words + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_u64_grid, dim3(zb ? zb : 1), dim3(256), 0, s, accs, acc_words);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, counters, 2 * kXcds);
    if (hub_tile == 512)
        launch_batch_bt<512>(batch_tile, descs, items, nums, accs, counters, grid, hub_grid, hub_chunk, s);
    else if (hub_tile == 1024)
        launch_batch_bt<1024>(batch_tile, descs, items, nums, accs, counters, grid, hub_grid, hub_chunk, s);
    else launch_batch_bt<2048>(batch_tile, descs, items, nums, accs, counters, grid, hub_grid, hub_chunk, s);
    return hipGetLastError();
}

hipError_t census_upload_table() {
    return hipMemcpyToSymbol(HIP_SYMBOL(c_table), kTable.t, sizeof(kTable.t));
}

namespace {

template <bool Tri>
void launch_bucket(int b, const census_args& L, uint64_t cnt, const census_config& cfg, unsigned int* counters,
                   hipStream_t s) {
    if (b == 0) {
        uint32_t grid = (uint32_t)std::min<uint64_t>((cnt + kLaneB - 1) / kLaneB, cfg.lane_blocks);
        size_t sh = Tri ? 0 : sizeof(unsigned long long) * lane_bins<kLaneB>::kWords;
        hipLaunchKernelGGL(k_census_lane<Tri>, dim3(grid), dim3(kLaneB), sh, s, L);
    } else if (b == 1) {
        const dim3 grid((uint32_t)std::min<uint64_t>(cnt, cfg.wave_blocks));
        unsigned int* c = counters + kXcds;
        if (cfg.wave_tile == 512) hipLaunchKernelGGL((k_census_wave<Tri, 512>), grid, dim3(kWaveB), 0, s, L, c);
        else if (cfg.wave_tile == 1024) hipLaunchKernelGGL((k_census_wave<Tri, 1024>), grid, dim3(kWaveB), 0, s, L, c);
        else hipLaunchKernelGGL((k_census_wave<Tri, 2048>), grid, dim3(kWaveB), 0, s, L, c);
    } else if (b == 2) {
        const dim3 grid((uint32_t)std::min<uint64_t>(cnt, cfg.group_blocks));
        unsigned int* c = counters + 2 * kXcds;
        if (cfg.group_size == 256) {
            if (cfg.group_tile == 2048) hipLaunchKernelGGL((k_census_group<Tri, 256, 2048>), grid, dim3(256), 0, s, L, c);
            else if (cfg.group_tile == 4096) hipLaunchKernelGGL((k_census_group<Tri, 256, 4096>), grid, dim3(256), 0, s, L, c);
            else hipLaunchKernelGGL((k_census_group<Tri, 256, 8192>), grid, dim3(256), 0, s, L, c);
        } else {
            if (cfg.group_tile == 2048) hipLaunchKernelGGL((k_census_group<Tri, 512, 2048>), grid, dim3(512), 0, s, L, c);
            else if (cfg.group_tile == 4096) hipLaunchKernelGGL((k_census_group<Tri, 512, 4096>), grid, dim3(512), 0, s, L, c);
            else hipLaunchKernelGGL((k_census_group<Tri, 512, 8192>), grid, dim3(512), 0, s, L, c);
        }
    }
}

// Task groups [g0, g1) of the ngroups, on the instance whose LDS holds the
// graph's groups (half-size groups: the smaller LDS).
template <bool Tri, uint32_t CH>
void launch_hub_ch(const census_args& L, const hub_task* tasks, uint32_t ntasks, uint32_t ngroups, uint32_t g0,
                   uint32_t g1, const census_config& cfg, unsigned int* c, hipStream_t s) {
    const dim3 grid((uint32_t)std::min<uint64_t>(g1 - g0, cfg.hub_blocks));
    if (cfg.hub_tile == 512)
        hipLaunchKernelGGL((k_census_hub<Tri, 512, CH>), grid, dim3(kHubB), 0, s, L, tasks, ntasks, ngroups, g0, g1, c);
    else if (cfg.hub_tile == 1024)
        hipLaunchKernelGGL((k_census_hub<Tri, 1024, CH>), grid, dim3(kHubB), 0, s, L, tasks, ntasks, ngroups, g0, g1, c);
    else
        hipLaunchKernelGGL((k_census_hub<Tri, 2048, CH>), grid, dim3(kHubB), 0, s, L, tasks, ntasks, ngroups, g0, g1, c);
}

template <bool Tri>
void launch_hub(const census_args& L, const hub_task* tasks, uint32_t ntasks, uint32_t ngroups, uint32_t g0,
                uint32_t g1, const census_config& cfg, unsigned int* counters, hipStream_t s) {
    unsigned int* c = counters + 3 * kXcds;
    if (L.hub_chunk <= kHubChunk / 2)
        launch_hub_ch<Tri, kHubChunk / 2>(L, tasks, ntasks, ngroups, g0, g1, cfg, c, s);
    else
        launch_hub_ch<Tri, kHubChunk>(L, tasks, ntasks, ngroups, g0, g1, cfg, c, s);
}

}  // namespace

hipError_t census_launch(const device_graph& g, const census_slices& sl, bool tri, const uint8_t* table,
                         unsigned long long* acc, unsigned int* counters, const census_config& cfg, hipStream_t s,
                         hipEvent_t* ev, hipStream_t side, hipEvent_t* fork) {
    if (!tile_supported(cfg.hub_tile, cfg.wave_tile, cfg.group_tile, cfg.group_size, 1024))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, acc, kNumClasses);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, counters, kBuckets * kXcds);
    const dyad_rec* recs = tri ? g.tri.edges.recs : g.dyads;
    const uint32_t* nbr = tri ? g.tri.fwd : g.nbr;
    // (the forward lists' half-size hub tasks when the graph has them)
    const bool fine = tri && g.tri.edges.fine_tasks != nullptr;
    const hub_task* tasks = fine ? g.tri.edges.fine_tasks : tri ? g.tri.edges.tasks : g.hub_tasks;
    const uint32_t ntasks = fine ? g.tri.edges.fine_n_tasks : tri ? g.tri.edges.n_tasks : g.n_hub_tasks;
    const uint32_t ngroups = fine ? g.tri.edges.fine_n_groups : tri ? g.tri.edges.n_groups : g.n_hub_groups;
    const uint32_t hg0 = std::min(sl.hub_g0, ngroups), hg1 = std::max(hg0, std::min(sl.hub_g1, ngroups));
    const uint64_t te0 = std::min<uint64_t>(sl.totals_begin, g.U);
    const uint64_t te1 = std::max(te0, std::min<uint64_t>(sl.totals_end, g.U));
    // (only when the hub kernel has more to stream than the totals pass)
    const bool beside = tri && side != nullptr && fork != nullptr && g.tri.edges.stream > g.U;
    if (tri) {
        // The totals pass (and the lane bucket after it) wait on memory and
        // the hub kernel on instruction issue: beside it, they use what the
        // hub kernel leaves.
        hipStream_t ts = s;
        if (beside) {
            hipError_t e = hipEventRecord(fork[0], s);
            if (e == hipSuccess) e = hipStreamWaitEvent(side, fork[0], 0);
            if (e != hipSuccess) return e;
            ts = side;
        }
        if (ev) (void)hipEventRecord(ev[2 * kBuckets], ts);
        if (te1 > te0) {
            uint32_t grid = (uint32_t)std::min<uint64_t>(
                (te1 - te0 + kTotalsPer * kLaneB - 1) / (kTotalsPer * kLaneB), beside ? cfg.side_blocks : cfg.lane_blocks);
            hipLaunchKernelGGL(k_census_totals, dim3(grid), dim3(kLaneB), 0, ts, g.nbr, g.owner, g.rinfo, g.tpre, te0,
                               te1, (uint64_t)g.n, table, acc);
        }
        if (ev) (void)hipEventRecord(ev[2 * kBuckets + 1], ts);
    }
    for (int b = 0; b < kBuckets; ++b) {
        uint64_t cnt = sl.end[b] > sl.begin[b] ? sl.end[b] - sl.begin[b] : 0;
        if (b == kBucketHub) cnt = hg1 - hg0;
        // beside the hub kernel, the lane bucket follows the totals pass on the side stream
        const hipStream_t bs = beside && b == 0 ? side : s;
        if (ev) (void)hipEventRecord(ev[2 * b], bs);
        if (cnt > 0) {
            census_args L{recs + sl.begin[b], (uint32_t)cnt, nbr, g.tpre, (uint64_t)g.n, acc, sl.u_lo, sl.u_hi,
                          table, fine ? kHubChunk / 2 : tri ? g.tri.edges.chunk : g.hub_chunk};
            if (b == kBucketHub) {
                L.dyads = recs;
                if (tri) launch_hub<true>(L, tasks, ntasks, ngroups, hg0, hg1, cfg, counters, s);
                else launch_hub<false>(L, tasks, ntasks, ngroups, hg0, hg1, cfg, counters, s);
            } else if (tri) {
                launch_bucket<true>(b, L, cnt, cfg, counters, bs);
            } else {
                launch_bucket<false>(b, L, cnt, cfg, counters, bs);
            }
        }
        if (ev) (void)hipEventRecord(ev[2 * b + 1], bs);
    }
    if (beside) {
        hipError_t e = hipEventRecord(fork[1], side);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, fork[1], 0);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace tc
