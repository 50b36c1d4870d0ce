// Graph build on the device: canonicalise arcs, sort, merge direction flags,
// CSR of undirected neighbours with two direction bits per entry, prefix
// counts of the direction bits, and the bucketed canonical-dyad task records.
//
// Follows the thesis's input model (section "Triad Census Algorithm"): a strict
// digraph G = [V, E] with E a set of ordered pairs and N(u) the undirected
// neighbourhood; and its adjacency-array (CRS) representation (section
// "Graph Data Structures").  Canonical dyads are the connected pairs u < v; the
// bucket key |N(u)| + |N(v)| - 2 is the workload estimate of the
// "Canonical Dyad (uniform distr.)" task-queue generation.
#include "tc_build.h"

#include <algorithm>
#include <vector>

namespace tc {

namespace {

constexpr int kT = 256;            // threads per block for build kernels
constexpr int kI = 8;              // items per thread
constexpr int kTile = kT * kI;     // 2048 items per block

inline uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + kTile - 1) / kTile); }

__device__ inline uint64_t lanemask_lt() {
    return (1ull << __lane_id()) - 1ull;
}

// ---- block-wide exclusive scan of one uint64 per thread (256 threads) ----
__device__ uint64_t block_exclusive_scan(uint64_t x, uint64_t* sh_warp /*[4]*/, uint64_t* block_total) {
    const int lane = __lane_id();
    const int wid = threadIdx.x >> 6;
    uint64_t incl = x;
    for (int off = 1; off < 64; off <<= 1) {
        uint64_t y = __shfl_up((unsigned long long)incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) sh_warp[wid] = incl;
    __syncthreads();
    uint64_t base = 0, tot = 0;
    for (int w = 0; w < kT / 64; ++w) {
        if (w < wid) base += sh_warp[w];
        tot += sh_warp[w];
    }
    __syncthreads();
    if (block_total) *block_total = tot;
    return base + incl - x;
}

__global__ __launch_bounds__(kT) void k_scan_reduce(const uint64_t* __restrict__ in, uint64_t n,
                                                     uint64_t* __restrict__ sums) {
    __shared__ uint64_t sh[kT / 64];
    uint64_t base = (uint64_t)blockIdx.x * kTile, s = 0;
    for (int k = 0; k < kI; ++k) {
        uint64_t i = base + (uint64_t)k * kT + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint64_t tot;
    block_exclusive_scan(s, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// single block: exclusive scan of sums[0..nb) in place, total to *total
__global__ __launch_bounds__(kT) void k_scan_spine(uint64_t* __restrict__ sums, uint64_t nb,
                                                    uint64_t* __restrict__ total) {
    __shared__ uint64_t sh[kT / 64];
    __shared__ uint64_t vals[kTile];
    uint64_t carry = 0;
    for (uint64_t base = 0; base < nb; base += kTile) {
        for (int k = 0; k < kI; ++k) {
            uint64_t i = base + (uint64_t)k * kT + threadIdx.x;
            vals[k * kT + threadIdx.x] = i < nb ? sums[i] : 0;
        }
        __syncthreads();
        uint64_t loc[kI], s = 0;
        for (int k = 0; k < kI; ++k) { loc[k] = s; s += vals[threadIdx.x * kI + k]; }
        uint64_t tot;
        uint64_t ex = block_exclusive_scan(s, sh, &tot);
        for (int k = 0; k < kI; ++k) vals[threadIdx.x * kI + k] = carry + ex + loc[k];
        __syncthreads();
        for (int k = 0; k < kI; ++k) {
            uint64_t i = base + (uint64_t)k * kT + threadIdx.x;
            if (i < nb) sums[i] = vals[k * kT + threadIdx.x];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kT) void k_scan_apply(const uint64_t* in, uint64_t* out, uint64_t n,
                                                    const uint64_t* __restrict__ sums) {
    __shared__ uint64_t sh[kT / 64];
    __shared__ uint64_t vals[kTile];
    uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (int k = 0; k < kI; ++k) {
        uint64_t i = base + (uint64_t)k * kT + threadIdx.x;
        vals[k * kT + threadIdx.x] = i < n ? in[i] : 0;
    }
    __syncthreads();
    uint64_t loc[kI], s = 0;
    for (int k = 0; k < kI; ++k) { loc[k] = s; s += vals[threadIdx.x * kI + k]; }
    uint64_t ex = block_exclusive_scan(s, sh, nullptr);
    uint64_t off = sums[blockIdx.x];
    for (int k = 0; k < kI; ++k) vals[threadIdx.x * kI + k] = off + ex + loc[k];
    __syncthreads();
    for (int k = 0; k < kI; ++k) {
        uint64_t i = base + (uint64_t)k * kT + threadIdx.x;
        if (i < n) out[i] = vals[k * kT + threadIdx.x];
    }
}

// ---- canonicalise: two keys per arc (one per orientation) -----------------
// key = owner << (bits + 2) | w << 2 | flag, flag 1 = owner->w, 2 = w->owner.
// Loops and bad ids become the sentinel (all sort bits set), which sorts last.
__global__ __launch_bounds__(kT) void k_canon(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                               uint64_t m, int32_t n, uint32_t bits, uint64_t* __restrict__ keys,
                                               unsigned long long* __restrict__ counters) {
    const uint64_t sentinel = (1ull << (2 * bits + 2)) - 1ull;
    uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    bool loop = false, bad = false;
    if (i < m) {
        int32_t s = src[i], d = dst[i];
        bad = s < 0 || s >= n || d < 0 || d >= n;
        loop = !bad && s == d;
        if (bad || loop) {
            keys[2 * i] = sentinel;
            keys[2 * i + 1] = sentinel;
        } else {
            keys[2 * i] = ((uint64_t)s << (bits + 2)) | ((uint64_t)d << 2) | 1ull;
            keys[2 * i + 1] = ((uint64_t)d << (bits + 2)) | ((uint64_t)s << 2) | 2ull;
        }
    }
    uint64_t nb = __ballot(bad), nl = __ballot(loop);
    if (__lane_id() == 0) {
        if (nb) atomicAdd(&counters[0], (unsigned long long)__popcll(nb));
        if (nl) atomicAdd(&counters[1], (unsigned long long)__popcll(nl));
    }
}

// ---- LSD radix sort, 8-bit digits starting at bit 2 ----------------------
__global__ __launch_bounds__(kT) void k_radix_hist(const uint64_t* __restrict__ keys, uint64_t count,
                                                    uint32_t shift, uint64_t* __restrict__ hist, uint32_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (int k = 0; k < kI; ++k) {
        uint64_t i = base + (uint64_t)k * kT + threadIdx.x;
        if (i < count) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: items are taken in index order (round r covers indices
// base + r*256 + t); a key's destination is the global offset of its digit in
// this block plus the number of equal digits before it inside the block.
__global__ __launch_bounds__(kT) void k_radix_scatter(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                       uint64_t count, uint32_t shift,
                                                       const uint64_t* __restrict__ offsets, uint32_t nblocks) {
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[kT / 64][256];
    __shared__ uint64_t goff[256];
    const int wid = threadIdx.x >> 6;
    running[threadIdx.x] = 0;
    goff[threadIdx.x] = offsets[(uint64_t)threadIdx.x * nblocks + blockIdx.x];
    for (int w = 0; w < kT / 64; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (int r = 0; r < kI; ++r) {
        uint64_t i = base + (uint64_t)r * kT + threadIdx.x;
        bool valid = i < count;
        uint64_t key = valid ? in[i] : 0;
        uint32_t dg = (uint32_t)((key >> shift) & 255u);
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot((dg >> b) & 1u);
            peers &= ((dg >> b) & 1u) ? bb : ~bb;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        bool leader = valid && (peers & lanemask_lt()) == 0;
        if (leader) wcnt[wid][dg] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t before = running[dg];
            for (int w = 0; w < wid; ++w) before += wcnt[w][dg];
            out[goff[dg] + before + rank] = key;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kT / 64; ++w) { add += wcnt[w][threadIdx.x]; wcnt[w][threadIdx.x] = 0; }
        running[threadIdx.x] += add;
        __syncthreads();
    }
}

// ---- unique (owner, w) pairs with OR-ed direction flags --------------------
__global__ __launch_bounds__(kT) void k_heads(const uint64_t* __restrict__ keys, uint64_t count,
                                               uint64_t* __restrict__ heads) {
    uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (i < count) heads[i] = (i == 0 || (keys[i] >> 2) != (keys[i - 1] >> 2)) ? 1ull : 0ull;
}

__global__ __launch_bounds__(kT) void k_emit(const uint64_t* __restrict__ keys, uint64_t count, uint32_t bits,
                                              const uint64_t* __restrict__ heads_in, const uint64_t* __restrict__ uidx,
                                              uint32_t* __restrict__ nbr, uint32_t* __restrict__ owner,
                                              unsigned long long* __restrict__ deg,
                                              unsigned long long* __restrict__ counters) {
    uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    bool dup = false;
    if (i < count && heads_in[i]) {
        uint64_t k = keys[i];
        uint32_t f = (uint32_t)(k & 3u);
        uint32_t seen1 = (f & 1u), seen2 = (f >> 1);
        for (uint64_t j = i + 1; j < count && (keys[j] >> 2) == (k >> 2); ++j) {
            uint32_t g = (uint32_t)(keys[j] & 3u);
            if ((g & 1u) && seen1) dup = true;
            if ((g & 2u) && seen2) dup = true;
            seen1 |= g & 1u;
            seen2 |= g >> 1;
            f |= g;
        }
        uint32_t w = (uint32_t)((k >> 2) & ((1ull << bits) - 1ull));
        uint32_t o = (uint32_t)(k >> (bits + 2));
        uint64_t e = uidx[i];
        nbr[e] = (w << 2) | f;
        owner[e] = o;
        atomicAdd(&deg[o], 1ull);
    }
    uint64_t nd = __ballot(dup);
    if (__lane_id() == 0 && nd) atomicAdd(&counters[2], (unsigned long long)__popcll(nd));
}

__global__ __launch_bounds__(kT) void k_type_bits(const uint32_t* __restrict__ nbr, uint64_t U,
                                                   uint64_t* __restrict__ t) {
    uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (i < U) {
        uint32_t f = nbr[i] & 3u;
        t[i] = (uint64_t)(f & 1u) | ((uint64_t)(f >> 1) << 32);
    }
}

// Per row: its bounds and the direction-bit prefix counts at its end.
__global__ __launch_bounds__(kT) void k_row_info(const int64_t* __restrict__ row_ptr, int32_t n,
                                                 const uint64_t* __restrict__ tpre, uint4* __restrict__ rinfo) {
    int32_t x = (int32_t)(blockIdx.x * kT + threadIdx.x);
    if (x < n) {
        const uint64_t rb = (uint64_t)row_ptr[x], re = (uint64_t)row_ptr[x + 1], t = tpre[re];
        rinfo[x] = make_uint4((uint32_t)rb, (uint32_t)re, (uint32_t)t, (uint32_t)(t >> 32));
    }
}

// degree statistics: max degree, sum of squares
__global__ __launch_bounds__(kT) void k_deg_stats(const int64_t* __restrict__ row_ptr, int32_t n,
                                                   unsigned long long* __restrict__ counters) {
    int32_t v = (int32_t)(blockIdx.x * kT + threadIdx.x);
    unsigned long long d = 0;
    if (v < n) d = (unsigned long long)(row_ptr[v + 1] - row_ptr[v]);
    unsigned long long sq = d * d, mx = d;
    for (int off = 32; off > 0; off >>= 1) {
        sq += __shfl_xor(sq, off, 64);
        unsigned long long o = __shfl_xor(mx, off, 64);
        mx = o > mx ? o : mx;
    }
    if (__lane_id() == 0) {
        atomicAdd(&counters[3], sq);
        atomicMax(&counters[4], mx);
    }
}

// ---- dyads: buckets, stable partition, hub tasks --------------------------
// Every connected pair is emitted once.  A pair whose larger degree is at
// least t_hub is a hub dyad, emitted from its anchor's row (the endpoint of
// larger degree, ties to the larger id), so the hub bucket is anchor-major;
// any other pair is emitted from the row of its smaller id (u-major) into the
// lane / wave / group bucket by k = |N(u)| + |N(v)| - 2.
// Bucket of entry e of an adjacency view.  Dyad view (tri = 0): the dyad is
// emitted once, from its first vertex, or from its anchor in the hub bucket.
// Forward view (tri = 1): every entry is one oriented edge and is emitted,
// unless one of the two forward lists is empty (no shared vertex possible).
// Hub: the longer of the two rows reaches t_hub; the anchor is the endpoint
// with the longer row (ties to the larger id).
__device__ inline int rec_bucket(const uint32_t* nbr, const uint32_t* owner, const int64_t* row_ptr,
                                 uint64_t e, uint64_t U, const bucket_params& bp, int tri, uint64_t* cost,
                                 uint64_t* stream, uint32_t* anchor) {
    if (e >= U) return kBuckets;
    const uint32_t o = owner[e], w = nbr[e] >> 2;
    const uint64_t d_o = (uint64_t)(row_ptr[o + 1] - row_ptr[o]), d_w = (uint64_t)(row_ptr[w + 1] - row_ptr[w]);
    if (tri && (d_o == 0 || d_w == 0)) return kBuckets;
    *cost = d_o + d_w;
    if ((d_o > d_w ? d_o : d_w) >= bp.t_hub) {
        const bool o_anchor = d_o > d_w || (d_o == d_w && o > w);
        if (!tri && !o_anchor) return kBuckets;
        *stream = o_anchor ? d_w : d_o;
        *anchor = o_anchor ? o : w;
        return kBucketHub;
    }
    if (!tri && !(o < w)) return kBuckets;
    const uint64_t k = tri ? d_o + d_w : d_o + d_w - 2;
    return k < bp.t0 ? 0 : (k < bp.t1 ? 1 : 2);
}

__global__ __launch_bounds__(kT) void k_dyad_count(const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ owner,
                                                    const int64_t* __restrict__ row_ptr, uint64_t U, bucket_params bp,
                                                    int tri, uint64_t* __restrict__ counts, uint32_t nblocks,
                                                    unsigned int* __restrict__ hubcnt,
                                                    unsigned long long* __restrict__ counters) {
    __shared__ uint32_t c[kBuckets];
    __shared__ unsigned long long cost_sh[kBuckets];
    __shared__ unsigned long long stream_sh;
    __shared__ uint32_t mutual_sh;
    if (threadIdx.x < kBuckets) { c[threadIdx.x] = 0; cost_sh[threadIdx.x] = 0; }
    if (threadIdx.x == 0) { mutual_sh = 0; stream_sh = 0; }
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * kTile;
    uint32_t my[kBuckets] = {0, 0, 0, 0}, mut = 0;
    unsigned long long mycost[kBuckets] = {0, 0, 0, 0}, mystream = 0;
    for (int k = 0; k < kI; ++k) {
        uint64_t e = base + (uint64_t)k * kT + threadIdx.x;
        uint64_t cost = 0, stream = 0;
        uint32_t anchor = 0;
        int b = rec_bucket(nbr, owner, row_ptr, e, U, bp, tri, &cost, &stream, &anchor);
        if (b < kBuckets) {
            my[b]++;
            mycost[b] += cost;
            mut += ((nbr[e] & 3u) == 3u) ? 1u : 0u;
            if (b == kBucketHub) {
                mystream += stream;
                atomicAdd(&hubcnt[anchor], 1u);
            }
        }
    }
    for (int b = 0; b < kBuckets; ++b) {
        if (my[b]) atomicAdd(&c[b], my[b]);
        if (mycost[b]) atomicAdd(&cost_sh[b], mycost[b]);
    }
    if (mut) atomicAdd(&mutual_sh, mut);
    if (mystream) atomicAdd(&stream_sh, mystream);
    __syncthreads();
    if (threadIdx.x < kBuckets) {
        counts[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = c[threadIdx.x];
        if (cost_sh[threadIdx.x]) atomicAdd(&counters[8 + threadIdx.x], cost_sh[threadIdx.x]);
    }
    if (threadIdx.x == 0 && mutual_sh) atomicAdd(&counters[5], (unsigned long long)mutual_sh);
    if (threadIdx.x == 0 && stream_sh) atomicAdd(&counters[12], stream_sh);
}

__device__ inline uint32_t find_in_row(const uint32_t* nbr, uint32_t lo, uint32_t hi, uint32_t x) {
    // first position in [lo, hi) whose vertex is >= x
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if ((nbr[mid] >> 2) < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Writes the records.  Lane / wave / group records keep the entry order of the
// view (u-major for dyads) through a stable per-bucket ranking.  Hub records
// of the dyad view come from their anchor's row and so are anchor-major in
// entry order; hub records of the forward view may come from either endpoint
// and are placed in their anchor's run (rec_off) through a per-anchor cursor.
__global__ __launch_bounds__(kT) void k_dyad_scatter(const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ owner,
                                                      const int64_t* __restrict__ row_ptr, uint64_t U, bucket_params bp,
                                                      int tri, const uint64_t* __restrict__ offsets, uint32_t nblocks,
                                                      const uint64_t* __restrict__ rec_off,
                                                      unsigned int* __restrict__ cursor, uint64_t hub_begin,
                                                      dyad_rec* __restrict__ out) {
    __shared__ uint32_t running[kBuckets];
    __shared__ uint32_t wcnt[kT / 64][kBuckets];
    __shared__ uint64_t goff[kBuckets];
    const int wid = threadIdx.x >> 6;
    if (threadIdx.x < kBuckets) {
        running[threadIdx.x] = 0;
        goff[threadIdx.x] = offsets[(uint64_t)threadIdx.x * nblocks + blockIdx.x];
    }
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (int r = 0; r < kI; ++r) {
        uint64_t e = base + (uint64_t)r * kT + threadIdx.x;
        uint64_t cost = 0, stream = 0;
        uint32_t anchor = 0;
        int b = rec_bucket(nbr, owner, row_ptr, e, U, bp, tri, &cost, &stream, &anchor);
        uint32_t rank = 0;
        for (int q = 0; q < kBuckets; ++q) {
            uint64_t mask = __ballot(b == q);
            if (b == q) rank = (uint32_t)__popcll(mask & lanemask_lt());
            if (__lane_id() == 0) wcnt[wid][q] = (uint32_t)__popcll(mask);
        }
        __syncthreads();
        if (b < kBuckets) {
            uint32_t before = running[b];
            for (int w = 0; w < wid; ++w) before += wcnt[w][b];
            const uint32_t o = owner[e], x = nbr[e] >> 2;
            const uint32_t u = o < x ? o : x, v = o < x ? x : o;
            dyad_rec rec;
            rec.bu = (uint32_t)row_ptr[u];
            rec.eu = (uint32_t)row_ptr[u + 1];
            rec.bv = (uint32_t)row_ptr[v];
            rec.ev = (uint32_t)row_ptr[v + 1];
            rec.u = u;
            if (tri) {
                const uint32_t fo = nbr[e] & 3u;
                const uint32_t fuv = o == u ? fo : ((fo & 1u) << 1) | (fo >> 1);
                rec.iv = 0;
                rec.iu = 0;
                rec.vf = (v << 2) | fuv;
            } else {
                if (o == u) {
                    rec.iv = (uint32_t)e;
                    rec.iu = find_in_row(nbr, rec.bv, rec.ev, u);
                } else {
                    rec.iu = (uint32_t)e;
                    rec.iv = find_in_row(nbr, rec.bu, rec.eu, v);
                }
                rec.vf = nbr[rec.iv];   // (v << 2) | f_uv
            }
            if (tri && b == kBucketHub)
                out[hub_begin + rec_off[anchor] + atomicAdd(&cursor[anchor], 1u)] = rec;
            else
                out[goff[b] + before + rank] = rec;
        }
        __syncthreads();
        if (threadIdx.x < kBuckets) {
            uint32_t add = 0;
            for (int w = 0; w < kT / 64; ++w) add += wcnt[w][threadIdx.x];
            running[threadIdx.x] += add;
        }
        __syncthreads();
    }
}

// Forward lists: flag the entries whose vertex follows the row's owner in
// degree order, compact them (order kept, so rows stay sorted by id), and read
// each row's start off the scanned flags.
__global__ __launch_bounds__(kT) void k_fwd_flag(const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ owner,
                                                  const int64_t* __restrict__ row_ptr, uint64_t U,
                                                  uint64_t* __restrict__ flag) {
    const uint64_t e = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= U) return;
    const uint32_t o = owner[e], w = nbr[e] >> 2;
    const int64_t d_o = row_ptr[o + 1] - row_ptr[o], d_w = row_ptr[w + 1] - row_ptr[w];
    flag[e] = (d_w > d_o || (d_w == d_o && w > o)) ? 1u : 0u;
}

__global__ __launch_bounds__(kT) void k_fwd_emit(const uint32_t* __restrict__ nbr, const uint32_t* __restrict__ owner,
                                                  uint64_t U, const uint64_t* __restrict__ pos,
                                                  uint32_t* __restrict__ fwd, uint32_t* __restrict__ fwd_owner) {
    const uint64_t e = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= U || pos[e + 1] == pos[e]) return;
    fwd[pos[e]] = nbr[e];
    fwd_owner[pos[e]] = owner[e];
}

__global__ __launch_bounds__(kT) void k_fwd_ptr(const int64_t* __restrict__ row_ptr, int32_t n,
                                                 const uint64_t* __restrict__ pos, int64_t* __restrict__ fwd_ptr) {
    const int64_t x = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (x <= n) fwd_ptr[x] = (int64_t)pos[row_ptr[x]];
}

// Hub tasks: the hub records of anchor row h are contiguous, starting at
// row_off[h] inside the hub bucket; they are cut into runs of kHubChunk.
// Tasks of anchors whose row is longer than `big_row` are placed first (they
// are the longest), the others after them: `big` selects which of the two
// classes this pass counts.
__global__ __launch_bounds__(kT) void k_hub_ntasks(const unsigned int* __restrict__ hubcnt, int32_t n,
                                                    const int64_t* __restrict__ row_ptr, uint64_t* __restrict__ ntask,
                                                    uint64_t big_row, int big, uint32_t chunk,
                                                    unsigned long long* __restrict__ counters) {
    int32_t h = (int32_t)(blockIdx.x * kT + threadIdx.x);
    unsigned long long staged = 0;
    if (h < n) {
        const uint64_t d = (uint64_t)(row_ptr[h + 1] - row_ptr[h]);
        uint64_t t = (hubcnt[h] + chunk - 1) / chunk;
        if ((d > big_row) != (big != 0)) t = 0;
        ntask[h] = t;
        staged = t * (unsigned long long)d;
    }
    for (int off = 32; off > 0; off >>= 1) staged += __shfl_xor(staged, off, 64);
    if (counters && __lane_id() == 0 && staged) atomicAdd(&counters[13], staged);
}

__global__ __launch_bounds__(kT) void k_hub_emit(const unsigned int* __restrict__ hubcnt, int32_t n,
                                                  const int64_t* __restrict__ row_ptr, const uint64_t* __restrict__ rec_off,
                                                  const uint64_t* __restrict__ task_off, uint64_t task_base, uint64_t big_row,
                                                  int big, uint32_t chunk, uint64_t hub_begin,
                                                  hub_task* __restrict__ tasks) {
    int32_t h = (int32_t)(blockIdx.x * kT + threadIdx.x);
    if (h >= n) return;
    if (((uint64_t)(row_ptr[h + 1] - row_ptr[h]) > big_row) != (big != 0)) return;
    const uint64_t c = hubcnt[h], base = hub_begin + rec_off[h], t0 = task_base + task_off[h];
    for (uint64_t j = 0; j * chunk < c; ++j) {
        hub_task t;
        t.begin = (uint32_t)(base + j * chunk);
        t.end = (uint32_t)(base + (c < (j + 1) * chunk ? c : (j + 1) * chunk));
        t.anchor = (uint32_t)h;
        t.group = 0;
        tasks[t0 + j] = t;
    }
}

// Groups of consecutive hub tasks that one workgroup runs with a single LDS
// tile: each window of kHubGroupTasks tasks is cut greedily before a task whose
// records would take the group past `chunk` or whose anchor row would take
// the group's rows past `tile` entries (a row longer than that stays alone).
// Without goff, counts the groups of every window into gcount; with goff (the
// scanned counts), stores the first task of each group in tasks[g].group.
__global__ __launch_bounds__(kT) void k_hub_group(hub_task* __restrict__ tasks, const dyad_rec* __restrict__ recs,
                                                  uint64_t ntasks, const uint64_t* __restrict__ goff,
                                                  uint64_t* __restrict__ gcount, uint32_t tile, uint32_t chunk) {
    const uint64_t w = (uint64_t)blockIdx.x * kT + threadIdx.x;
    const uint64_t t0 = w * kHubGroupTasks;
    if (t0 >= ntasks) return;
    const uint32_t nt = (uint32_t)(ntasks - t0 < kHubGroupTasks ? ntasks - t0 : kHubGroupTasks);
    uint32_t starts[kHubGroupTasks];
    uint32_t ng = 0, gs = 0, sr = 0, se = 0;
    for (uint32_t j = 0; j < nt; ++j) {
        const uint32_t b = tasks[t0 + j].begin, e = tasks[t0 + j].end, a = tasks[t0 + j].anchor;
        const dyad_rec r0 = recs[b];
        const uint32_t l = r0.u == a ? r0.eu - r0.bu : r0.ev - r0.bv, r = e - b;
        if (j > gs && (l > tile || sr + r > chunk || se + l > tile)) {
            starts[ng++] = gs;
            gs = j;
            sr = 0;
            se = 0;
        }
        sr += r;
        se += l;
    }
    starts[ng++] = gs;
    if (goff == nullptr) {
        gcount[w] = ng;
    } else {
        for (uint32_t k = 0; k < ng; ++k) tasks[goff[w] + k].group = (uint32_t)t0 + starts[k];
    }
}

__global__ void k_u32_to_u64(const unsigned int* __restrict__ a, uint64_t* __restrict__ b, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline uint32_t grid1(uint64_t n) { return (uint32_t)((n + kT - 1) / kT); }

}  // namespace

hipError_t fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid1(n)), dim3(kT), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t scan_exclusive_u64(const uint64_t* in, uint64_t* out, uint64_t count, uint64_t* total_dev,
                              hipStream_t s) {
    if (count == 0) {
        return total_dev ? fill_u64(total_dev, 1, 0, s) : hipSuccess;
    }
    uint32_t nb = blocks_for(count);
    uint64_t* sums = nullptr;
    hipError_t e = hipMallocAsync((void**)&sums, sizeof(uint64_t) * (nb + 1), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kT), 0, s, in, count, sums);
    hipLaunchKernelGGL(k_scan_spine, dim3(1), dim3(kT), 0, s, sums, (uint64_t)nb, total_dev);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kT), 0, s, in, out, count, (const uint64_t*)sums);
    e = hipGetLastError();
    hipError_t e2 = hipFreeAsync(sums, s);
    return e != hipSuccess ? e : e2;
}

// Sorts `count` keys on bits [2, 2 + sort_bits); result in *keys (buffers swapped as needed).
static hipError_t radix_sort(uint64_t** keys, uint64_t** tmp, uint64_t count, uint32_t sort_bits, hipStream_t s) {
    if (count <= 1) return hipSuccess;
    uint32_t nb = blocks_for(count);
    uint64_t* hist = nullptr;
    hipError_t e = hipMallocAsync((void**)&hist, sizeof(uint64_t) * 256ull * nb, s);
    if (e != hipSuccess) return e;
    for (uint32_t shift = 2; shift < 2 + sort_bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kT), 0, s, *keys, count, shift, hist, nb);
        e = scan_exclusive_u64(hist, hist, 256ull * nb, nullptr, s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kT), 0, s, *keys, *tmp, count, shift,
                           (const uint64_t*)hist, nb);
        if ((e = hipGetLastError()) != hipSuccess) break;
        std::swap(*keys, *tmp);
    }
    hipError_t e2 = hipFreeAsync(hist, s);
    return e != hipSuccess ? e : e2;
}

static uint32_t bit_width_u32(uint32_t x) {
    uint32_t b = 0;
    while (x) { ++b; x >>= 1; }
    return b;
}

#define TRY(x) do { hipError_t _e = (x); if (_e != hipSuccess) { err = _e; goto done; } } while (0)

build_status build_graph_device(int32_t n, int64_t m, const int32_t* src_dev, const int32_t* dst_dev,
                                const bucket_params& bp, hipStream_t s, device_graph* g) {
    build_status st{};
    hipError_t err = hipSuccess;
    uint64_t *keys = nullptr, *tmp = nullptr, *heads = nullptr, *uidx = nullptr, *degs = nullptr;
    unsigned long long* counters = nullptr;
    unsigned long long hc[kCounters] = {0};
    uint64_t valid = 0, U = 0;
    uint32_t bits = bit_width_u32((uint32_t)n);
    uint64_t total_keys = 2ull * (uint64_t)m;

    *g = device_graph{};
    g->n = n;
    TRY(hipMallocAsync((void**)&counters, sizeof(unsigned long long) * kCounters, s));
    TRY(fill_u64((uint64_t*)counters, kCounters, 0, s));
    TRY(hipMalloc((void**)&g->row_ptr, sizeof(int64_t) * ((size_t)n + 1)));
    if (total_keys > 0) {
        TRY(hipMallocAsync((void**)&keys, sizeof(uint64_t) * total_keys, s));
        TRY(hipMallocAsync((void**)&tmp, sizeof(uint64_t) * total_keys, s));
        hipLaunchKernelGGL(k_canon, dim3(grid1((uint64_t)m)), dim3(kT), 0, s, src_dev, dst_dev, (uint64_t)m, n, bits,
                           keys, counters);
        TRY(hipGetLastError());
        TRY(hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
        st.bad_ids = (int64_t)hc[0];
        st.self_loops = (int64_t)hc[1];
        if (st.bad_ids) goto done;
        TRY(radix_sort(&keys, &tmp, total_keys, 2 * bits, s));
        valid = total_keys - 2ull * hc[1];
    }
    // unique entries
    if (valid > 0) {
        TRY(hipMallocAsync((void**)&heads, sizeof(uint64_t) * valid, s));
        TRY(hipMallocAsync((void**)&uidx, sizeof(uint64_t) * (valid + 1), s));
        hipLaunchKernelGGL(k_heads, dim3(grid1(valid)), dim3(kT), 0, s, keys, valid, heads);
        TRY(hipGetLastError());
        TRY(scan_exclusive_u64(heads, uidx, valid, uidx + valid, s));
        TRY(hipMemcpyAsync(&U, uidx + valid, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
    }
    if (U >= (1ull << 32)) { st.too_large = true; goto done; }
    g->U = U;
    TRY(hipMallocAsync((void**)&degs, sizeof(uint64_t) * ((size_t)n + 1), s));
    TRY(fill_u64(degs, (uint64_t)n + 1, 0, s));
    TRY(hipMalloc((void**)&g->nbr, sizeof(uint32_t) * (U + kRowPad)));
    TRY(hipMalloc((void**)&g->owner, sizeof(uint32_t) * (U ? U : 1)));
    TRY(hipMalloc((void**)&g->tpre, sizeof(uint64_t) * (U + 1)));
    if (valid > 0) {
        hipLaunchKernelGGL(k_emit, dim3(grid1(valid)), dim3(kT), 0, s, keys, valid, bits, heads, uidx, g->nbr,
                           g->owner, (unsigned long long*)degs, counters);
        TRY(hipGetLastError());
    }
    TRY(scan_exclusive_u64(degs, (uint64_t*)g->row_ptr, (uint64_t)n + 1, nullptr, s));
    // direction-bit prefix counts
    if (U > 0) {
        hipLaunchKernelGGL(k_type_bits, dim3(grid1(U)), dim3(kT), 0, s, g->nbr, U, g->tpre);
        TRY(hipGetLastError());
    }
    TRY(scan_exclusive_u64(g->tpre, g->tpre, U, g->tpre + U, s));
    TRY(hipMalloc((void**)&g->rinfo, sizeof(uint4) * ((size_t)n + 1)));
    if (n > 0) {
        hipLaunchKernelGGL(k_row_info, dim3(grid1((uint64_t)n)), dim3(kT), 0, s, (const int64_t*)g->row_ptr, n,
                           (const uint64_t*)g->tpre, g->rinfo);
        TRY(hipGetLastError());
    }
    if (n > 0) {
        hipLaunchKernelGGL(k_deg_stats, dim3(grid1((uint64_t)n)), dim3(kT), 0, s, g->row_ptr, n, counters);
        TRY(hipGetLastError());
    }
    TRY(hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, s));
    {
        uint64_t tot = 0;
        TRY(hipMemcpyAsync(&tot, g->tpre + U, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
        st.arcs_kept = (int64_t)(tot & 0xffffffffull);
        st.duplicates = (int64_t)hc[2];
        st.sum_d2 = hc[3];
        st.max_degree = (int64_t)hc[4];
    }
    TRY(bucket_dyads(g, bp, s));
    st.ok = true;
done:
    if (keys) (void)hipFreeAsync(keys, s);
    if (tmp) (void)hipFreeAsync(tmp, s);
    if (heads) (void)hipFreeAsync(heads, s);
    if (uidx) (void)hipFreeAsync(uidx, s);
    if (degs) (void)hipFreeAsync(degs, s);
    if (counters) (void)hipFreeAsync(counters, s);
    (void)hipStreamSynchronize(s);
    st.hip = err;
    if (!st.ok) {
        free_device_graph(g);
    }
    return st;
}

// Cuts the hub records of each anchor (contiguous from hub_begin + rec_off[h])
// into tasks of at most `chunk` records, anchors whose rows span several LDS
// tiles first, and the tasks into groups (k_hub_group).  The staged entries
// of the tasks are added to ctr[13] unless ctr is null.
static hipError_t cut_hub_tasks(const unsigned int* hubcnt, int32_t n, const int64_t* row_ptr,
                                const uint64_t* rec_off, uint64_t* tmp64, uint64_t hub_begin, const dyad_rec* recs,
                                const bucket_params& bp, uint32_t chunk, unsigned long long* ctr, hipStream_t s,
                                hub_task** tasks_out, uint32_t* ntasks_out, uint32_t* ngroups_out) {
    hipError_t err = hipSuccess;
    uint64_t *task_off = nullptr, *gcount = nullptr;
    hub_task* tasks = nullptr;
    uint64_t part[2] = {0, 0}, ntasks = 0, ngroups = 0, windows = 0;
    TRY(hipMallocAsync((void**)&task_off, sizeof(uint64_t) * ((size_t)n + 1), s));
    for (int big = 1; big >= 0; --big) {
        hipLaunchKernelGGL(k_hub_ntasks, dim3(grid1((uint64_t)n)), dim3(kT), 0, s, hubcnt, n, row_ptr, tmp64,
                           (uint64_t)bp.hub_tile, big, chunk, ctr);
        TRY(hipGetLastError());
        TRY(scan_exclusive_u64(tmp64, task_off, (uint64_t)n, task_off + n, s));
        TRY(hipMemcpyAsync(&part[big], task_off + n, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
    }
    ntasks = part[1] + part[0];
    TRY(hipMalloc((void**)&tasks, sizeof(hub_task) * (ntasks ? ntasks : 1)));
    for (int big = 1; big >= 0; --big) {
        hipLaunchKernelGGL(k_hub_ntasks, dim3(grid1((uint64_t)n)), dim3(kT), 0, s, hubcnt, n, row_ptr, tmp64,
                           (uint64_t)bp.hub_tile, big, chunk, (unsigned long long*)nullptr);
        TRY(hipGetLastError());
        TRY(scan_exclusive_u64(tmp64, task_off, (uint64_t)n, task_off + n, s));
        hipLaunchKernelGGL(k_hub_emit, dim3(grid1((uint64_t)n)), dim3(kT), 0, s, hubcnt, n, row_ptr, rec_off, task_off,
                           big ? (uint64_t)0 : part[1], (uint64_t)bp.hub_tile, big, chunk, hub_begin, tasks);
        TRY(hipGetLastError());
    }
    windows = (ntasks + kHubGroupTasks - 1) / kHubGroupTasks;
    TRY(hipMallocAsync((void**)&gcount, sizeof(uint64_t) * (windows + 1), s));
    hipLaunchKernelGGL(k_hub_group, dim3(grid1(windows)), dim3(kT), 0, s, tasks, recs, ntasks,
                       (const uint64_t*)nullptr, gcount, bp.hub_tile, chunk);
    TRY(hipGetLastError());
    TRY(scan_exclusive_u64(gcount, gcount, windows, gcount + windows, s));
    hipLaunchKernelGGL(k_hub_group, dim3(grid1(windows)), dim3(kT), 0, s, tasks, recs, ntasks,
                       (const uint64_t*)gcount, (uint64_t*)nullptr, bp.hub_tile, chunk);
    TRY(hipGetLastError());
    TRY(hipMemcpyAsync(&ngroups, gcount + windows, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    *tasks_out = tasks;
    tasks = nullptr;
    *ntasks_out = (uint32_t)ntasks;
    *ngroups_out = (uint32_t)ngroups;
done:
    if (tasks) (void)hipFree(tasks);
    if (task_off) (void)hipFreeAsync(task_off, s);
    if (gcount) (void)hipFreeAsync(gcount, s);
    return err;
}

// Buckets the entries of one adjacency view (nbr / owner / row_ptr over U
// entries and n rows) into `out`: records, hub tasks and the per-bucket sums.
static hipError_t bucket_records(const uint32_t* nbr, const uint32_t* owner, const int64_t* row_ptr, uint64_t U,
                                 int32_t n, int tri, const bucket_params& bp, hipStream_t s, rec_set* out,
                                 uint64_t* mutual) {
    hipError_t err = hipSuccess;
    uint64_t* counts = nullptr;
    unsigned long long* counters = nullptr;
    unsigned int *hubcnt = nullptr, *cursor = nullptr;
    uint64_t *rec_off = nullptr, *tmp64 = nullptr;
    unsigned long long hc[kCounters] = {0};
    uint64_t off_host[kBuckets + 1] = {0, 0, 0, 0, 0};
    uint64_t total = 0;
    const uint32_t nb = blocks_for(U ? U : 1);
    if (out->recs) (void)hipFree(out->recs);
    if (out->tasks) (void)hipFree(out->tasks);
    if (out->fine_tasks) (void)hipFree(out->fine_tasks);
    *out = rec_set{};
    TRY(hipMallocAsync((void**)&counters, sizeof(unsigned long long) * kCounters, s));
    TRY(fill_u64((uint64_t*)counters, kCounters, 0, s));
    TRY(hipMallocAsync((void**)&counts, sizeof(uint64_t) * ((size_t)kBuckets * nb + 1), s));
    TRY(hipMallocAsync((void**)&hubcnt, sizeof(unsigned int) * ((size_t)n + 2), s));
    TRY(fill_u64((uint64_t*)hubcnt, ((uint64_t)n + 2) / 2, 0, s));
    TRY(hipMallocAsync((void**)&rec_off, sizeof(uint64_t) * ((size_t)n + 1), s));
    TRY(hipMallocAsync((void**)&tmp64, sizeof(uint64_t) * ((size_t)n + 1), s));
    if (tri) {
        TRY(hipMallocAsync((void**)&cursor, sizeof(unsigned int) * ((size_t)n + 2), s));
        TRY(fill_u64((uint64_t*)cursor, ((uint64_t)n + 2) / 2, 0, s));
    }
    hipLaunchKernelGGL(k_dyad_count, dim3(nb), dim3(kT), 0, s, nbr, owner, row_ptr, U, bp, tri, counts, nb, hubcnt,
                       counters);
    TRY(hipGetLastError());
    TRY(scan_exclusive_u64(counts, counts, (uint64_t)kBuckets * nb, counts + (uint64_t)kBuckets * nb, s));
    // bucket starts: the scanned value at the first block of each bucket
    for (int b = 0; b < kBuckets; ++b)
        TRY(hipMemcpyAsync(&off_host[b], counts + (uint64_t)b * nb, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    TRY(hipMemcpyAsync(&off_host[kBuckets], counts + (uint64_t)kBuckets * nb, sizeof(uint64_t),
                       hipMemcpyDeviceToHost, s));
    // per anchor: offset of its run of hub records
    if (n > 0) {
        hipLaunchKernelGGL(k_u32_to_u64, dim3(grid1((uint64_t)n)), dim3(kT), 0, s, hubcnt, tmp64, (uint64_t)n);
        TRY(hipGetLastError());
        TRY(scan_exclusive_u64(tmp64, rec_off, (uint64_t)n, rec_off + n, s));
    }
    TRY(hipStreamSynchronize(s));
    total = off_host[kBuckets];
    for (int b = 0; b <= kBuckets; ++b) out->off[b] = off_host[b];
    TRY(hipMalloc((void**)&out->recs, sizeof(dyad_rec) * (total ? total : 1)));
    if (total > 0) {
        hipLaunchKernelGGL(k_dyad_scatter, dim3(nb), dim3(kT), 0, s, nbr, owner, row_ptr, U, bp, tri,
                           (const uint64_t*)counts, nb, (const uint64_t*)rec_off, cursor, out->off[kBucketHub],
                           out->recs);
        TRY(hipGetLastError());
    }
    // hub tasks and their groups: of kHubChunk records (the set batched
    // launches run), and for a forward-list hub bucket of kHubSplitRecords
    // records or more also of half as many (the set a single census runs)
    if (out->off[kBucketHub + 1] > out->off[kBucketHub] && n > 0) {
        const bool fine = tri && out->off[kBucketHub + 1] - out->off[kBucketHub] >= kHubSplitRecords;
        TRY(cut_hub_tasks(hubcnt, n, row_ptr, rec_off, tmp64, out->off[kBucketHub], out->recs, bp, kHubChunk,
                          counters, s, &out->tasks, &out->n_tasks, &out->n_groups));
        if (fine)
            TRY(cut_hub_tasks(hubcnt, n, row_ptr, rec_off, tmp64, out->off[kBucketHub], out->recs, bp, kHubChunk / 2,
                              counters + 1, s, &out->fine_tasks, &out->fine_n_tasks, &out->fine_n_groups));
    }
    TRY(hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    for (int b = 0; b < kBuckets; ++b) out->cost[b] = hc[8 + b];
    if (mutual) *mutual = hc[5];
    out->stream = hc[12];
    out->staged = hc[13];
    out->fine_staged = hc[14];
done:
    if (counts) (void)hipFreeAsync(counts, s);
    if (counters) (void)hipFreeAsync(counters, s);
    if (hubcnt) (void)hipFreeAsync(hubcnt, s);
    if (cursor) (void)hipFreeAsync(cursor, s);
    if (rec_off) (void)hipFreeAsync(rec_off, s);
    if (tmp64) (void)hipFreeAsync(tmp64, s);
    (void)hipStreamSynchronize(s);
    return err;
}

static void free_forward(forward_lists* t) {
    if (t->fwd) (void)hipFree(t->fwd);
    if (t->fwd_owner) (void)hipFree(t->fwd_owner);
    if (t->fwd_ptr) (void)hipFree(t->fwd_ptr);
    if (t->edges.recs) (void)hipFree(t->edges.recs);
    if (t->edges.tasks) (void)hipFree(t->edges.tasks);
    if (t->edges.fine_tasks) (void)hipFree(t->edges.fine_tasks);
    *t = forward_lists{};
}

// Forward lists of g (degree order), built once per graph.
static hipError_t build_forward(device_graph* g, hipStream_t s) {
    hipError_t err = hipSuccess;
    uint64_t* pos = nullptr;
    const uint64_t U = g->U;
    const int32_t n = g->n;
    forward_lists& t = g->tri;
    TRY(hipMalloc((void**)&t.fwd_ptr, sizeof(int64_t) * ((size_t)n + 1)));
    TRY(hipMallocAsync((void**)&pos, sizeof(uint64_t) * (U + 1), s));
    if (U > 0) {
        hipLaunchKernelGGL(k_fwd_flag, dim3(grid1(U)), dim3(kT), 0, s, g->nbr, g->owner, g->row_ptr, U, pos);
        TRY(hipGetLastError());
    }
    TRY(scan_exclusive_u64(pos, pos, U, pos + U, s));
    TRY(hipMemcpyAsync(&t.entries, pos + U, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    TRY(hipMalloc((void**)&t.fwd, sizeof(uint32_t) * (t.entries + kRowPad)));
    TRY(hipMalloc((void**)&t.fwd_owner, sizeof(uint32_t) * (t.entries ? t.entries : 1)));
    if (U > 0) {
        hipLaunchKernelGGL(k_fwd_emit, dim3(grid1(U)), dim3(kT), 0, s, g->nbr, g->owner, U, (const uint64_t*)pos,
                           t.fwd, t.fwd_owner);
        TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_fwd_ptr, dim3(grid1((uint64_t)n + 1)), dim3(kT), 0, s, g->row_ptr, n,
                       (const uint64_t*)pos, t.fwd_ptr);
    TRY(hipGetLastError());
done:
    if (pos) (void)hipFreeAsync(pos, s);
    (void)hipStreamSynchronize(s);
    return err;
}

hipError_t bucket_dyads(device_graph* g, const bucket_params& bp, hipStream_t s) {
    rec_set d;
    d.recs = g->dyads;
    d.tasks = g->hub_tasks;
    g->dyads = nullptr;
    g->hub_tasks = nullptr;
    g->n_hub_tasks = 0;
    g->n_hub_groups = 0;
    uint64_t mutual = 0;
    hipError_t err = bucket_records(g->nbr, g->owner, g->row_ptr, g->U, g->n, 0, bp, s, &d, &mutual);
    g->dyads = d.recs;
    g->hub_tasks = d.tasks;
    if (err != hipSuccess) return err;
    g->n_hub_tasks = d.n_tasks;
    g->n_hub_groups = d.n_groups;
    g->hub_chunk = d.chunk;
    g->p = d.off[kBuckets];
    for (int b = 0; b <= kBuckets; ++b) g->bucket_off[b] = d.off[b];
    for (int b = 0; b < kBuckets; ++b) g->bucket_cost[b] = d.cost[b];
    g->mutual = mutual;
    g->hub_stream = d.stream;
    g->hub_staged = d.staged;
    g->bp = bp;
    if (!bp.tri) {
        free_forward(&g->tri);
        return hipSuccess;
    }
    if (!g->tri.fwd_ptr) {
        err = build_forward(g, s);
        if (err != hipSuccess) {
            free_forward(&g->tri);
            return err;
        }
    }
    forward_lists& t = g->tri;
    err = bucket_records(t.fwd, t.fwd_owner, t.fwd_ptr, t.entries, g->n, 1, bp, s, &t.edges, nullptr);
    if (err != hipSuccess) free_forward(&g->tri);
    return err;
}

#undef TRY

void free_device_graph(device_graph* g) {
    free_forward(&g->tri);
    if (g->row_ptr) (void)hipFree(g->row_ptr);
    if (g->nbr) (void)hipFree(g->nbr);
    if (g->owner) (void)hipFree(g->owner);
    if (g->tpre) (void)hipFree(g->tpre);
    if (g->rinfo) (void)hipFree(g->rinfo);
    if (g->dyads) (void)hipFree(g->dyads);
    if (g->hub_tasks) (void)hipFree(g->hub_tasks);
    int32_t n = g->n;
    *g = device_graph{};
    g->n = n;
}

uint64_t device_graph_bytes(const device_graph& g) {
    uint64_t b = sizeof(int64_t) * ((uint64_t)g.n + 1) + (sizeof(uint32_t) * 2 + sizeof(uint64_t)) * g.U +
                 sizeof(uint32_t) * kRowPad + sizeof(uint4) * ((uint64_t)g.n + 1) +
                 sizeof(uint64_t) + sizeof(dyad_rec) * g.p + sizeof(hub_task) * (uint64_t)g.n_hub_tasks;
    if (g.tri.fwd_ptr)
        b += sizeof(int64_t) * ((uint64_t)g.n + 1) + sizeof(uint32_t) * (2 * g.tri.entries + kRowPad) +
             sizeof(dyad_rec) * g.tri.edges.off[kBuckets] +
             sizeof(hub_task) * ((uint64_t)g.tri.edges.n_tasks + g.tri.edges.fine_n_tasks);
    return b;
}

}  // namespace tc
