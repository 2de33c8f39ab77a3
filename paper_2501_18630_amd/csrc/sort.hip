// Tile binning and (view, tile, depth, id) ordering.
//
// Sec. 3.2 composites the primitives that overlap a pixel in depth order.
// Instead of one wide radix sort of (tile | depth) keys over all pairs, the
// order is built in two narrow stable sorts:
//   1. radix-sort the visible (view, splat) records by the fp32 bits of
//      their depth (32 bits; the first pass reads the visibility bits, depth
//      keys and packed tile rectangles of all records in place, the others
//      the P visible ones; each record's rectangle travels with it, so the
//      emission below reads it in depth order without a gather); stability
//      keeps equal depths in record order, i.e. by splat index within a view;
//   2. emit one (global tile id, record) pair per overlapped tile, walking
//      the records in depth order, and radix-sort the pairs by tile id only
//      (ceil(log2 tiles) bits, over K pairs); stability keeps the depth
//      order inside each tile.
// The result is exactly the lexicographic (view, tile, depth bits, splat id)
// order, at 2-3 narrow passes over the K pairs instead of 6-7 wide ones.
//
// The radix sort is a classic LSD sort with 8- or 9-bit digits: per-block digit
// histograms (upsweep), a scan of each digit's counts over the blocks plus
// the digit totals, and a stable scatter (downsweep) that ranks each block's keys
// with wave ballots and per-wave digit counts in LDS (no LDS atomics, one
// barrier per phase) and writes them out digit-contiguous.  Element counts
// are read from device memory, so the whole pipeline runs without a host
// round trip and can be captured in a graph.
#include <mutex>
#include <type_traits>

#include "dbs_internal.h"

namespace dbs {

namespace {

struct Count {
    const uint32_t *dev;  // if non-null, n = min(*dev, host)
    int64_t host;
    __device__ inline int64_t get() const
    {
        if (dev) {
            int64_t d = *dev;
            return d < host ? d : host;
        }
        return host;
    }
};

__device__ inline uint64_t lanemask_lt()
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Exclusive scan of one value per thread across a block of NT threads.
template <int NT = kSortThreads>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_tmp /*[NT/kWave + 1]*/, uint32_t *total)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) s_tmp[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int k = 0; k < NT / kWave; ++k) {
            uint32_t c = s_tmp[k];
            s_tmp[k] = acc;
            acc += c;
        }
        s_tmp[NT / kWave] = acc;
    }
    __syncthreads();
    uint32_t r = s_tmp[w] + x - v;
    if (total) *total = s_tmp[NT / kWave];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- scans

// Exclusive scan of row[0..n) in place by one workgroup of NT threads, each
// taking 16 consecutive entries of a tile of 16 NT (four 16-byte loads and
// stores; row must start on 16 bytes); returns the total.
template <int NT>
__device__ uint32_t scan_in_place(uint32_t *row, int64_t n, uint32_t *s_tmp /*[NT/kWave + 1]*/)
{
    uint32_t carry = 0;
    for (int64_t base = 0; base < n; base += 16 * NT) {  // uniform
        const int64_t e0 = base + (int64_t)threadIdx.x * 16;
        const bool whole = e0 + 16 <= n;
        uint32_t v[16], acc = 0;
        if (whole) {
            const uint4 *src = reinterpret_cast<const uint4 *>(row + e0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 u = src[q];
                v[4 * q] = u.x;
                v[4 * q + 1] = u.y;
                v[4 * q + 2] = u.z;
                v[4 * q + 3] = u.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = e0 + k < n ? row[e0 + k] : 0u;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) acc += v[k];
        uint32_t total;
        uint32_t pre = carry + block_exclusive_scan<NT>(acc, s_tmp, &total);
        uint32_t o[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            o[k] = pre;
            pre += v[k];
        }
        if (whole) {
            uint4 *dst = reinterpret_cast<uint4 *>(row + e0);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = make_uint4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (e0 + k < n) row[e0 + k] = o[k];
        }
        carry += total;
    }
    return carry;
}

// Single-block exclusive scan of partials[0..nb), in place.  With `items`
// set, only the ceil(*items / per_block) partials of blocks that hold items
// are scanned (the grid before it was sized for the capacity).
__global__ __launch_bounds__(1024) void scan_partials_kernel(uint32_t *partials, int64_t nb,
                                                             const uint32_t *items = nullptr, int per_block = 1)
{
    __shared__ uint32_t s_tmp[1024 / kWave + 1];
    if (items) {
        const int64_t used = ((int64_t)*items + per_block - 1) / per_block;
        if (used < nb) nb = used;
    }
    scan_in_place<1024>(partials, nb, s_tmp);
}

// Exclusive scan of each digit's row of the digit-major histogram of a radix
// pass, over the blocks that hold keys, in place; workgroup d also writes the
// digit's total.  Rows start on 16 bytes (the row stride is a multiple of 4).
constexpr int kDigitScanThreads = 1024;
__global__ __launch_bounds__(kDigitScanThreads) void scan_digits_kernel(uint32_t *hist, int64_t hstride, Count cnt,
                                                                        uint32_t *totals)
{
    __shared__ uint32_t s_tmp[kDigitScanThreads / kWave + 1];
    const int64_t n = cnt.get();
    const int64_t nb_used = (n + kSortTile - 1) / kSortTile;
    const uint32_t total = scan_in_place<kDigitScanThreads>(hist + (int64_t)blockIdx.x * hstride, nb_used, s_tmp);
    if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

// ---------------------------------------------------------------- radix sort

// Digit match across the wave: mask of valid lanes holding digit d (RB bits).
// Per bit: m = the bit sign-extended (0 or all ones), its ballot B, and each
// half of the mask keeps the lanes whose bit agrees, mask & ~(B ^ m) — one
// three-input bitwise instruction per half, four VALU per bit in all.
template <int RB>
__device__ inline uint64_t match_digit(uint32_t d, bool valid)
{
    const uint64_t v = __ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        uint32_t m = (uint32_t)((int32_t)(d << (31 - b)) >> 31);
        asm volatile("" : "+v"(m));  // keeps the ballot's compare on m (not a second shift of d)
        const uint64_t bal = __ballot(m != 0u);
        lo &= ~((uint32_t)bal ^ m);
        hi &= ~((uint32_t)(bal >> 32) ^ m);
    }
    return ((uint64_t)hi << 32) | lo;
}

// Block b sorts elements [b * kSortTile, (b + 1) * kSortTile); inside it wave w
// owns the contiguous 1024 elements from w * 1024, item k of lane l being
// element w * 1024 + k * 64 + l, so that (wave, item, lane) is element order.
// Digit counts are kept per wavefront in LDS.  The upsweep only counts, and
// adds with LDS atomics (one instruction per item, no cross-lane matching).
// The downsweep needs each element's rank among equal digits in element
// order, so it matches digits across the wave and one leader lane per
// distinct digit updates the count with a plain read-add-write: the leaders
// of one wave hold distinct digits, and no other wave touches the wave's row.
// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b on XCD
// b % 8) and every XCD has its own L2.  Chunk c of the keys is given to
// workgroup b with c = (b % 8) * (nb / 8) + b / 8 (up to the last nb % 8), so
// that each XCD sorts a contiguous range of chunks: the digit-major histogram
// entries a workgroup writes, and the boundaries of the digit runs it
// scatters, then share cache lines with its neighbours on the same XCD
// instead of being written back piecewise by several L2s.
__device__ __forceinline__ int64_t xcd_chunk(int64_t b, int64_t nb)
{
    const int64_t full = nb & ~(int64_t)7;
    return b < full ? (b & 7) * (full >> 3) + (b >> 3) : b;
}

__device__ __forceinline__ int64_t sort_elem(int64_t block_base, int w, int k, int lane)
{
    return block_base + (int64_t)w * (kSortItems * kWave) + (int64_t)k * kWave + lane;
}

// Tile rectangle of a record's pixel box (tile sides 2^lw x 2^lh;
// boxes are clipped to the image, so the coordinates are not negative).
struct TileRect {
    int tx0, ty0, w, h;
};
__device__ __forceinline__ TileRect tile_rect(short4 b, int lw, int lh)
{
    TileRect r;
    r.tx0 = b.x >> lw;
    r.ty0 = b.z >> lh;
    r.w = (b.y >> lw) - r.tx0 + 1;
    r.h = (b.w >> lh) - r.ty0 + 1;
    return r;
}

// The packed tile rectangle (pack_tile_rect) as a TileRect.
__device__ __forceinline__ TileRect unpack_rect(uint32_t p)
{
    TileRect r;
    r.tx0 = (int)(p & 1023u);
    r.ty0 = (int)((p >> 10) & 1023u);
    r.w = (int)((p >> 20) & 63u) + 1;
    r.h = (int)(p >> 26) + 1;
    return r;
}

// The first pass of the depth sort reads the preprocess's output in place
// (no compaction pass): chunk c is the 4096 splats [j 4096, (j + 1) 4096) of
// view v, c = v nbv + j; an element is valid where its visibility bit is set
// (ntiles > 0; the bits past n are zero), its key is the record's depth bits,
// its value the record v n + i and its carried word the record's packed tile
// rectangle.  Chunks in order are records in order, so the pass is the
// stable sort of the visible records in record order.
static_assert(kSortTile == 4096, "a chunk is one block of the visibility bit rows");
struct VisSrc {
    const BinsHeader *bh = nullptr;  // n_rec == 0: the buffers do not match, nothing is valid
    const uint32_t *visbits = nullptr, *depth = nullptr, *rect = nullptr;
    int64_t n = 0, vstride = 0, nbv = 0, nbc = 0;
};

// Wavefront w's slice of chunk c: item k of lane l is splat i0 + 64 k + l.
struct VisSlice {
    const uint32_t *bits, *dep, *rct;
    int64_t i0, rec0, n;
    bool ok;
    __device__ VisSlice(const VisSrc &vs, int64_t c, int w_)
    {
        const int w = __builtin_amdgcn_readfirstlane(w_);  // uniform: the bit words are scalar loads
        const int64_t v = c / vs.nbv;
        i0 = (c - v * vs.nbv) * kSortTile + (int64_t)w * (kSortItems * kWave);
        n = vs.n;
        rec0 = v * n + i0;
        bits = vs.visbits + v * vs.vstride + (i0 >> 5);
        dep = vs.depth + v * n;
        rct = vs.rect + v * n;
        ok = vs.bh->n_rec != 0;
    }
    // visibility bits of item k's 64 splats (two words, 8-byte aligned);
    // read only when ok
    __device__ uint64_t word(int k) const { return *reinterpret_cast<const uint64_t *>(bits + 2 * k); }
    // depth bits of item k of this lane (clamped in range; used only where valid)
    __device__ uint32_t key(int k, int lane) const
    {
        const int64_t i = i0 + (int64_t)k * kWave + lane;
        return dep[i < n ? i : n - 1];
    }
    // packed tile rectangle of item k of this lane (clamped likewise)
    __device__ uint32_t rect(int k, int lane) const
    {
        const int64_t i = i0 + (int64_t)k * kWave + lane;
        return rct[i < n ? i : n - 1];
    }
};

template <int RB, bool VIS = false>
__global__ __launch_bounds__(kSortThreads) void radix_upsweep_kernel(const uint32_t *keys, Count cnt, int shift,
                                                                     int width, uint32_t *hist, int64_t hstride,
                                                                     VisSrc vs = {})
{
    // UC count rows per wave, lane l adding into row l % UC: equal digits of
    // one wave then collide UC times less, and the odd row stride puts the
    // rows' copies of one digit in different banks
    constexpr int NW = kSortThreads / kWave, RADIX = 1 << RB, DPT = RADIX / kSortThreads, UC = 4;
    constexpr int STRIDE = RADIX + 1, ROWS = NW * UC;
    __shared__ uint32_t s_cnt[ROWS * STRIDE];
    const uint32_t dmask = (1u << width) - 1u;
    const int t = threadIdx.x, w = t / kWave, lane = t & (kWave - 1);
    const int64_t n = VIS ? vs.nbc * kSortTile : cnt.get();
    const int64_t nb_used = (n + kSortTile - 1) / kSortTile;  // the grid is sized for the capacity
    const int64_t chunk = (int64_t)blockIdx.x < nb_used ? xcd_chunk(blockIdx.x, nb_used) : (int64_t)blockIdx.x;
    const int64_t base = chunk * kSortTile;
    for (int i = t; i < ROWS * STRIDE; i += kSortThreads) s_cnt[i] = 0;
    __syncthreads();
    if constexpr (VIS) {
        const VisSlice vsl(vs, chunk, w);
        uint32_t d[kSortItems];
        if (vsl.ok) {  // uniform; on a buffer mismatch nothing is read and nothing counts
#pragma unroll
            for (int k = 0; k < kSortItems; ++k) {  // all loads in flight before any counting
                const uint32_t key = vsl.key(k, lane);
                d[k] = (vsl.word(k) >> lane) & 1ull ? (key >> shift) & dmask : RADIX;
            }
        } else {
#pragma unroll
            for (int k = 0; k < kSortItems; ++k) d[k] = RADIX;
        }
        // an invalid item is not counted: about half the items of a view are
        // invisible, and adding them all into one padding entry serialised
        // the wave's atomics on that address
        uint32_t *row = s_cnt + (w * UC + (lane & (UC - 1))) * STRIDE;
#pragma unroll
        for (int k = 0; k < kSortItems; ++k)
            if (d[k] < RADIX) atomicAdd(&row[d[k]], 1u);
    } else {
        // compiled twice: for a full chunk (all but the last) without bounds tests
        auto count_chunk = [&](auto full_tag) {
            constexpr bool FULL = decltype(full_tag)::value;
            uint32_t d[kSortItems];
#pragma unroll
            for (int k = 0; k < kSortItems; ++k) {  // all loads in flight before any counting
                const int64_t e = sort_elem(base, w, k, lane);
                d[k] = FULL || e < n ? (keys[e] >> shift) & dmask : RADIX;
            }
            uint32_t *row = s_cnt + (w * UC + (lane & (UC - 1))) * STRIDE;
#pragma unroll
            for (int k = 0; k < kSortItems; ++k)
                if (FULL || d[k] < RADIX) atomicAdd(&row[d[k]], 1u);
        };
        if (base + kSortTile <= n)
            count_chunk(std::integral_constant<bool, true>{});
        else if (base < n)
            count_chunk(std::integral_constant<bool, false>{});
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        const int dd = q * kSortThreads + t;
        uint32_t tot = 0;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) tot += s_cnt[r * STRIDE + dd];
        hist[(int64_t)dd * hstride + chunk] = tot;
    }
}

// The output offset of digit d of this chunk is the digit's base (the
// exclusive scan of the digit totals) plus the chunk's entry of the
// per-digit scanned histogram.  The last pass writes no keys (they are not
// needed afterwards).  AUX: the values are pairs (record, packed tile
// rectangle), moved as one 8-byte word; the VIS pass builds them from the
// record index and the preprocess's rectangles.  In the last pass, if ranges is set
// (a sort by the full key, ranges[] holding (~0, 0) before), each key's
// output range [start, end) is recorded in ranges[key]: a block's equal keys
// are contiguous in its LDS-sorted order and in the output, and the blocks'
// pieces of a key's range are merged with atomic min / max.
// LAST: the sort's last pass (values only; ranges).  With 8-bit digits and
// no carried word it is held to 128 VGPRs for a fourth wavefront per SIMD
// (measured faster there, not in the other 8-bit passes); 9-bit passes are
// held to 128 VGPRs with a 16-bit digit table for the same (the two passes
// of 18-bit tile keys over 346 M pairs 1929 + 1519 -> 1844 + 1493 us).
template <bool AUX>
using SortVal = std::conditional_t<AUX, uint2, uint32_t>;

template <int RB, bool VIS = false, bool LAST = false, bool AUX = false>
__global__ __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu((LAST && RB == 8 && !AUX) || RB == 9 ? 4 : 1))) void radix_downsweep_kernel(
    const uint32_t *__restrict__ keys_in, const SortVal<AUX> *__restrict__ vals_in, uint32_t *__restrict__ keys_out,
    SortVal<AUX> *__restrict__ vals_out, Count cnt, int shift, int width, const uint32_t *hist,
    const uint32_t *totals, int64_t hstride, uint2 *ranges, VisSrc vs = {})
{
    using VT = SortVal<AUX>;
    constexpr bool last = LAST;
    constexpr int NW = kSortThreads / kWave, RADIX = 1 << RB, DPT = RADIX / kSortThreads;
    __shared__ uint32_t s_keys[kSortTile];
    __shared__ VT s_vals[kSortTile];
    // per-wave digit counts, then per-wave offsets (below 4096); 16-bit where
    // a word is carried (three workgroups then fit in a CU's LDS) and with
    // 9-bit digits (four)
    using WH = std::conditional_t<AUX || RB == 9, uint16_t, uint32_t>;
    __shared__ WH s_wh[NW][RADIX];
    __shared__ uint32_t s_goff[RADIX];
    __shared__ uint32_t s_tmp[NW + 1];
    const uint32_t dmask = (1u << width) - 1u;

    const int64_t n = VIS ? vs.nbc * kSortTile : cnt.get();
    const int64_t nb_used = (n + kSortTile - 1) / kSortTile;  // the grid is sized for the capacity
    const int64_t chunk = (int64_t)blockIdx.x < nb_used ? xcd_chunk(blockIdx.x, nb_used) : (int64_t)blockIdx.x;
    const int64_t base = chunk * kSortTile;
    if (base >= n) return;  // uniform across the block
    const int t = threadIdx.x, w = t / kWave, lane = t & (kWave - 1);
    uint32_t cnt_vis = 0;  // VIS: the chunk's valid elements
    {   // thread t owns digits t * DPT .. t * DPT + DPT - 1
        uint32_t tot[DPT], sum = 0;
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            tot[q] = totals[t * DPT + q];
            sum += tot[q];
        }
        uint32_t st = block_exclusive_scan(sum, s_tmp, nullptr);
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            const int dd = t * DPT + q;
            s_goff[dd] = st + hist[(int64_t)dd * hstride + chunk];
            st += tot[q];
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) s_wh[ww][dd] = 0;
        }
    }
    __syncthreads();

    // Loads, ranking and the scatter into LDS, compiled twice: for a chunk
    // that is full (all but the last), without the per-item bounds tests.
    const bool full = !VIS && base + kSortTile <= n;  // uniform across the block
    auto sort_chunk = [&](auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        uint32_t key[kSortItems], rank[kSortItems];
        VT val[kSortItems];
        uint32_t vbits = 0;  // VIS: bit k set where item k is valid
        const uint64_t lt = lanemask_lt();
        if constexpr (VIS) {
            static_assert(AUX, "the first depth pass carries the tile rectangles");
            const VisSlice vsl(vs, chunk, w);
#pragma unroll
            for (int k = 0; k < kSortItems; ++k) {
                key[k] = 0u;
                val[k] = make_uint2((uint32_t)(vsl.rec0 + (int64_t)k * kWave + lane), 0u);
            }
            if (vsl.ok) {  // uniform; on a buffer mismatch nothing is read and nothing is valid
#pragma unroll
                for (int k = 0; k < kSortItems; ++k) {  // all loads in flight before the ranking
                    key[k] = vsl.key(k, lane);
                    vbits |= (uint32_t)((vsl.word(k) >> lane) & 1ull) << k;
                    val[k].y = vsl.rect(k, lane);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < kSortItems; ++k) {  // all loads in flight before the ranking
                const int64_t e = sort_elem(base, w, k, lane);
                key[k] = FULL || e < n ? keys_in[e] : 0u;
                val[k] = FULL || e < n ? vals_in[e] : VT{};
            }
        }
        auto item_valid = [&](int k) -> bool {
            if constexpr (VIS) return (vbits >> k) & 1u;
            return FULL || sort_elem(base, w, k, lane) < n;
        };
        // rank inside the wave: earlier items of this wave, then lower lanes of this item
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            const bool valid = item_valid(k);
            const uint32_t d = (key[k] >> shift) & dmask;
            const uint64_t peers = match_digit<RB>(d, valid);
            const uint32_t before = s_wh[w][d];
            if (valid && (peers & lt) == 0) s_wh[w][d] = (WH)(before + (uint32_t)__popcll(peers));
            rank[k] = before + (uint32_t)__popcll(peers & lt);
        }
        __syncthreads();
        {   // thread t owns digits t * DPT .. t * DPT + DPT - 1: s_wh[w][d] becomes
            // the LDS position of wave w's first item of digit d, s_goff[d] the
            // output offset minus digit d's first LDS position
            uint32_t c[DPT][NW], tot[DPT], sum = 0;
#pragma unroll
            for (int q = 0; q < DPT; ++q) {
                tot[q] = 0;
#pragma unroll
                for (int ww = 0; ww < NW; ++ww) {
                    c[q][ww] = s_wh[ww][t * DPT + q];
                    tot[q] += c[q][ww];
                }
                sum += tot[q];
            }
            uint32_t st = block_exclusive_scan(sum, s_tmp, &cnt_vis);
#pragma unroll
            for (int q = 0; q < DPT; ++q) {
                const int dd = t * DPT + q;
                s_goff[dd] -= st;
#pragma unroll
                for (int ww = 0; ww < NW; ++ww) {
                    s_wh[ww][dd] = (WH)st;
                    st += c[q][ww];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            if (item_valid(k)) {
                const uint32_t pos = s_wh[w][(key[k] >> shift) & dmask] + rank[k];
                s_keys[pos] = key[k];
                s_vals[pos] = val[k];
            }
        }
    };
    if (full)
        sort_chunk(std::integral_constant<bool, true>{});
    else
        sort_chunk(std::integral_constant<bool, false>{});
    __syncthreads();
    const int64_t cnt_blk = VIS ? (int64_t)cnt_vis : (n - base < kSortTile ? n - base : kSortTile);
    for (int j = t; j < cnt_blk; j += kSortThreads) {
        const uint32_t kk = s_keys[j];
        const uint32_t d = (kk >> shift) & dmask;
        const uint32_t o = s_goff[d] + (uint32_t)j;
        if (!last) keys_out[o] = kk;
        vals_out[o] = s_vals[j];
        if (last && ranges) {
            if (j == 0 || s_keys[j - 1] != kk) atomicMin(&ranges[kk].x, o);
            if (j == cnt_blk - 1 || s_keys[j + 1] != kk) atomicMax(&ranges[kk].y, o + 1);
        }
    }
}

int radix_passes(int bits) { return (bits + kMaxRadixBits - 1) / kMaxRadixBits; }

// Stable sort of (keys, vals) by key bits [bit_lo, bit_hi); ping-pongs
// between the a and b buffers and reports where the values ended up (the
// sorted keys are not kept: the last pass writes values only).  The bits are
// split into radix_passes() digits of at most kMaxRadixBits, as even as
// possible (17 bits: 9 + 8, not 8 + 8 + 1).  Each pass: per-chunk digit
// counts, a per-digit scan over the chunks (with the digit totals in
// `totals`, kMaxRadix entries), and the stable scatter.  ranges applies to
// the last pass (see radix_downsweep_kernel).  Values of type uint2 are
// (record, packed tile rectangle) pairs and take 8-bit digits only; with vis
// the first pass reads the elements in place (see VisSrc).
template <typename VT>
hipError_t radix_sort(uint32_t *ka, VT *va, uint32_t *kb, VT *vb, Count cnt, int bit_lo, int bit_hi,
                      uint32_t *hist, uint32_t *totals, hipStream_t s, bool *result_in_b, uint2 *ranges = nullptr,
                      const VisSrc *vis = nullptr)
{
    constexpr bool aux = std::is_same_v<VT, uint2>;
    const int bits = bit_hi - bit_lo, passes = radix_passes(bits);
    if (vis && (!aux || passes < 2 || bits > 8 * passes)) return hipErrorInvalidValue;  // 8-bit first pass, not the last
    if (aux && bits > 8 * passes) return hipErrorInvalidValue;
    bool in_b = false;
    int shift = bit_lo;
    for (int p = 0; p < passes; ++p) {
        const int width = (bits - (shift - bit_lo) + (passes - p) - 1) / (passes - p);
        const uint32_t *kin = in_b ? kb : ka;
        const VT *vin = in_b ? vb : va;
        uint32_t *kout = in_b ? ka : kb;
        VT *vout = in_b ? va : vb;
        const bool last = p == passes - 1;
        uint2 *rg = last ? ranges : nullptr;
        if constexpr (aux) {
            if (p == 0 && vis) {  // straight from the visibility bits, depth keys and tile rectangles
                const int64_t nb = vis->nbc, hs = hist_stride(nb);
                radix_upsweep_kernel<8, true><<<(unsigned)nb, kSortThreads, 0, s>>>(nullptr, cnt, shift, width,
                                                                                     hist, hs, *vis);
                scan_digits_kernel<<<1u << 8, kDigitScanThreads, 0, s>>>(hist, hs, Count{nullptr, nb * kSortTile},
                                                                         totals);
                radix_downsweep_kernel<8, true, false, true><<<(unsigned)nb, kSortThreads, 0, s>>>(
                    nullptr, nullptr, kout, vout, cnt, shift, width, hist, totals, hs, nullptr, *vis);
                in_b = !in_b;
                shift += width;
                continue;
            }
        }
        const int64_t nblocks = ceil_div(cnt.host > 0 ? cnt.host : 1, kSortTile);
        const int64_t hstride = hist_stride(nblocks);  // histogram rows start on 16 bytes
        if (width <= 8) {
            radix_upsweep_kernel<8><<<(unsigned)nblocks, kSortThreads, 0, s>>>(kin, cnt, shift, width, hist, hstride);
            scan_digits_kernel<<<1u << 8, kDigitScanThreads, 0, s>>>(hist, hstride, cnt, totals);
            if (last)
                radix_downsweep_kernel<8, false, true, aux><<<(unsigned)nblocks, kSortThreads, 0, s>>>(
                    kin, vin, kout, vout, cnt, shift, width, hist, totals, hstride, rg);
            else
                radix_downsweep_kernel<8, false, false, aux><<<(unsigned)nblocks, kSortThreads, 0, s>>>(
                    kin, vin, kout, vout, cnt, shift, width, hist, totals, hstride, rg);
        } else if constexpr (!aux) {
            radix_upsweep_kernel<9><<<(unsigned)nblocks, kSortThreads, 0, s>>>(kin, cnt, shift, width, hist, hstride);
            scan_digits_kernel<<<1u << 9, kDigitScanThreads, 0, s>>>(hist, hstride, cnt, totals);
            if (last)
                radix_downsweep_kernel<9, false, true><<<(unsigned)nblocks, kSortThreads, 0, s>>>(
                    kin, vin, kout, vout, cnt, shift, width, hist, totals, hstride, rg);
            else
                radix_downsweep_kernel<9><<<(unsigned)nblocks, kSortThreads, 0, s>>>(
                    kin, vin, kout, vout, cnt, shift, width, hist, totals, hstride, rg);
        }
        in_b = !in_b;
        shift += width;
    }
    *result_in_b = in_b;
    return hipGetLastError();
}

// ---------------------------------------------------------------- binning kernels

// The pair count was taken by the preprocess with its tile shape: binning
// with another shape, splat count or view count would emit a different
// number of pairs than the capacity check saw, so such a call bins nothing
// (overflow 2), as does a count above the capacity (overflow 1).
__global__ void finalize_counts_kernel(const ProjHeader *ph, BinsHeader *bh, int64_t n, int32_t n_views, int tw,
                                       int th, int64_t cap, uint32_t n_tiles, int32_t *overflow_out)
{
    if (threadIdx.x != 0) return;
    const bool match = ph->n == n && ph->n_views == n_views && ph->tile_w == tw && ph->tile_h == th;
    const int64_t vis = ph->counts[0], pairs = ph->counts[1];
    const int32_t ovf = !match ? 2 : (pairs > cap ? 1 : 0);
    bh->overflow = ovf;
    bh->n_rec = match ? (uint32_t)(n * n_views) : 0u;
    bh->n_vis = match ? (uint32_t)vis : 0u;
    bh->n_pairs = ovf ? 0u : (uint32_t)pairs;
    bh->n_tiles = n_tiles;
    bh->n_views = n_views;
    bh->tile_w = tw;
    bh->tile_h = th;
    bh->n = n;
    for (int k = 0; k < 4; ++k) bh->queue[k] = 0;
    if (overflow_out) *overflow_out = ovf;
}

// Blocks of 4096 records for the pair counts.
constexpr int kCompactItems = 16;
constexpr int kCompactTile = kSortThreads * kCompactItems;

// floor(x / d) for 32-bit x and a divisor d >= 2 fixed for the launch, from
// m = ceil(2^64 / d): x m / 2^64 exceeds x / d by less than 2^-32, which
// cannot carry it past the next integer.
struct Div32 {
    uint64_t m;
    bool one;  // d == 1
};
inline Div32 make_div32(uint32_t d)
{
    Div32 v;
    v.one = d <= 1;
    v.m = v.one ? 0 : (~0ull / d) + 1;  // floor((2^64 - 1) / d) + 1 = ceil(2^64 / d)
    return v;
}
__device__ __forceinline__ uint32_t div32(uint32_t x, const Div32 &d) { return d.one ? x : (uint32_t)__umul64hi(x, d.m); }

// Pair counts of the depth-ordered records: per block of 4096 records (16
// consecutive ones per thread) into block_sum, and per group of 256 records
// (one emission block) into group_sum.
__global__ __launch_bounds__(kSortThreads) void count_pairs_kernel(const BinsHeader *bh, const uint2 *sorted,
                                                                   const short4 *bbox, int lw, int lh,
                                                                   uint32_t *block_sum, uint32_t *group_sum)
{
    __shared__ uint32_t s_tmp[kSortThreads / kWave + 1];
    const int64_t nvis = bh->overflow ? 0 : (int64_t)bh->n_vis;
    const int64_t base = (int64_t)blockIdx.x * kCompactTile;
    if (base >= nvis) return;  // uniform; its sums are never read
    const int t = threadIdx.x;
    const int64_t e0 = base + (int64_t)t * kCompactItems;
    uint32_t cnt = 0;
    if (e0 + kCompactItems <= nvis) {
        // the packed rectangles first, with no branch between the loads; a
        // thread with an escaped rectangle (rare) then counts that one again
        // from its pixel box
        const uint4 *src = reinterpret_cast<const uint4 *>(sorted + e0);
        uint4 u[kCompactItems / 2];  // two (record, rectangle) pairs each
#pragma unroll
        for (int q = 0; q < kCompactItems / 2; ++q) u[q] = src[q];
        bool esc = false;
#pragma unroll
        for (int q = 0; q < kCompactItems / 2; ++q) {
            const TileRect r0 = unpack_rect(u[q].y), r1 = unpack_rect(u[q].w);
            cnt += (u[q].y != kRectEscape ? (uint32_t)(r0.w * r0.h) : 0u) +
                   (u[q].w != kRectEscape ? (uint32_t)(r1.w * r1.h) : 0u);
            esc |= u[q].y == kRectEscape || u[q].w == kRectEscape;
        }
        if (esc) {
#pragma unroll
            for (int q = 0; q < kCompactItems / 2; ++q) {
                if (u[q].y == kRectEscape) {
                    const TileRect r = tile_rect(bbox[u[q].x], lw, lh);
                    cnt += (uint32_t)(r.w * r.h);
                }
                if (u[q].w == kRectEscape) {
                    const TileRect r = tile_rect(bbox[u[q].z], lw, lh);
                    cnt += (uint32_t)(r.w * r.h);
                }
            }
        }
    } else {
        for (int q = 0; q < kCompactItems; ++q)
            if (e0 + q < nvis) {
                const uint2 u = sorted[e0 + q];
                const TileRect r = u.y != kRectEscape ? unpack_rect(u.y) : tile_rect(bbox[u.x], lw, lh);
                cnt += (uint32_t)(r.w * r.h);
            }
    }
    // groups of 256 records = 16 consecutive lanes
    uint32_t g = cnt;
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) g += __shfl_xor(g, off, 16);
    if ((t & 15) == 0) group_sum[(int64_t)blockIdx.x * 16 + (t >> 4)] = g;
    uint32_t total;
    block_exclusive_scan(cnt, s_tmp, &total);
    if (t == 0) block_sum[blockIdx.x] = total;
}

// Pair emission.  One block per 256 depth-ordered records: their tile counts
// are scanned in the block; the block's first pair is its 4096-record block's
// scanned offset plus the pairs of the groups before it.  Each wavefront
// writes a contiguous range of the block's pairs, 64 consecutive pairs per
// step (contiguous stores).  The record of each pair: the record holding the
// step's first pair (a binary search at a wavefront's first step, then carried
// over), plus the number of records that start at or before the pair within
// the step (their start positions are flagged in LDS and read back as one
// ballot).
__global__ __launch_bounds__(256) void emit_pairs_kernel(const BinsHeader *bh, const uint2 *sorted,
                                                         const short4 *bbox, const ViewDesc *views,
                                                         Div32 n, int lw, int lh, const uint32_t *block_sum,
                                                         const uint32_t *group_sum, uint32_t *pkeys,
                                                         uint32_t *pvals)
{
    __shared__ uint32_t s_off[257];
    __shared__ uint32_t s_rec[256], s_row0[256], s_tx[256];
    __shared__ uint2 s_w[256];  // (tile columns w, bits of the float 1 / w)
    __shared__ uint32_t s_tmp[kSortThreads / kWave + 1];
    __shared__ uint8_t s_flag[256 / kWave][kWave];
    const int64_t nvis = bh->overflow ? 0 : (int64_t)bh->n_vis;  // nothing is emitted on overflow
    const int64_t j0 = (int64_t)blockIdx.x * 256;
    if (j0 >= nvis) return;  // uniform
    const int cntb = nvis - j0 < 256 ? (int)(nvis - j0) : 256;
    const int t = threadIdx.x, w = t / kWave, lane = t & (kWave - 1);
    uint32_t cnt = 0;
    if (t < cntb) {
        const uint2 u = sorted[j0 + t];
        const uint32_t rec = u.x;
        const TileRect r = u.y != kRectEscape ? unpack_rect(u.y) : tile_rect(bbox[rec], lw, lh);
        const ViewDesc &V = views[div32(rec, n)];
        cnt = (uint32_t)(r.w * r.h);
        s_rec[t] = rec;
        s_row0[t] = (uint32_t)V.tile_offset + (uint32_t)(r.ty0 * V.tiles_x + r.tx0);
        s_tx[t] = (uint32_t)V.tiles_x;
        s_w[t] = make_uint2((uint32_t)r.w, __float_as_uint(__builtin_amdgcn_rcpf((float)r.w)));
    }
    uint32_t total;
    const uint32_t off = block_exclusive_scan(cnt, s_tmp, &total);
    uint64_t base = block_sum[blockIdx.x >> 4];
    for (unsigned gi = blockIdx.x & ~15u; gi < blockIdx.x; ++gi) base += group_sum[gi];
    if (t < cntb) s_off[t] = off;
    if (t == 0) s_off[cntb] = total;
    __syncthreads();
    const uint64_t cap = bh->n_pairs;  // pairs are only emitted below the binned count
    // the step range, the step's first pair and its record are wave-uniform
    // (scalar registers and loop control)
    const uint32_t tot_u = __builtin_amdgcn_readfirstlane(total);
    const uint32_t nsteps = (tot_u + kWave - 1) / kWave, per = (nsteps + 3) / 4;
    const uint32_t c0 = __builtin_amdgcn_readfirstlane(w) * per, c1 = c0 + per < nsteps ? c0 + per : nsteps;
    int r_cur = -1;
    const uint64_t upto = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);
    for (uint32_t c = c0; c < c1; ++c) {
        const uint32_t q0 = c * kWave;
        int r0;
        if (r_cur < 0) {  // the record holding pair q0
            int lo = 0, hi = cntb - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (__builtin_amdgcn_readfirstlane(s_off[mid]) <= q0) lo = mid; else hi = mid - 1;
            }
            r0 = lo;
        } else {
            r0 = (r_cur + 1 < cntb && __builtin_amdgcn_readfirstlane(s_off[r_cur + 1]) <= q0) ? r_cur + 1 : r_cur;
        }
        s_flag[w][lane] = 0;
        __builtin_amdgcn_wave_barrier();
        const int idx = r0 + 1 + lane;
        if (idx < cntb) {
            const uint32_t d = s_off[idx] - q0;
            if (d < (uint32_t)kWave) s_flag[w][d] = 1;
        }
        __builtin_amdgcn_wave_barrier();
        const uint64_t starts = __ballot(s_flag[w][lane] != 0);
        const int r = r0 + __popcll(starts & upto);
        const uint32_t q = q0 + lane;
        const uint64_t gp = base + q;
        if (q < total && gp < cap) {
            // (dy, dx) of the pair inside the record's tile rectangle: the quotient
            // from the float reciprocal is off by at most one (local < 2^22)
            const uint2 wrr = s_w[r];
            const uint32_t local = q - s_off[r], wr = wrr.x;
            uint32_t dy = (uint32_t)((float)local * __uint_as_float(wrr.y));
            int32_t rem = (int32_t)local - (int32_t)(dy * wr);
            const bool neg = rem < 0, big = rem >= (int32_t)wr;  // at most one holds
            dy = dy + (big ? 1u : 0u) - (neg ? 1u : 0u);
            rem += neg ? (int32_t)wr : (big ? -(int32_t)wr : 0);
            pkeys[gp] = s_row0[r] + dy * s_tx[r] + (uint32_t)rem;
            pvals[gp] = s_rec[r];
        }
        r_cur = __builtin_amdgcn_readlane(r, kWave - 1);
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t count, uint32_t value)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// Tile ranges before the last pass of the pair sort records them: (~0, 0),
// so that atomic min / max leave (first, last + 1) of each listed tile.
__global__ void fill_ranges_kernel(uint2 *ranges, int64_t n_tiles)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_tiles) ranges[i] = make_uint2(0xffffffffu, 0u);
}

// Heaviest tiles first, by an 8-bit cost class so that one radix pass sorts
// them: the pair count c itself below 16, above it 16 classes per octave
// (the leading five bits of c), with c capped at 0xffff (class 207); key =
// 255 - class, ties in tile order.  Also turns the range of a tile no pair
// reached, still (~0, 0), into (0, 0).
__global__ void tile_cost_keys_kernel(uint2 *ranges, int64_t n_tiles, uint32_t *keys, uint32_t *vals)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    uint2 r = ranges[t];
    if (r.x == 0xffffffffu) {
        r = make_uint2(0u, 0u);
        ranges[t] = r;
    }
    uint32_t c = r.y - r.x;
    c = c < 0xffffu ? c : 0xffffu;
    uint32_t cls = c;
    if (c >= 16u) {
        const int e = 31 - __builtin_clz(c);  // 4 .. 15
        cls = (uint32_t)(e - 3) * 16u + ((c >> (e - 4)) & 15u);
    }
    keys[t] = 255u - cls;
    vals[t] = (uint32_t)t;
}

int bits_for(int64_t count)
{
    int b = 0;
    while (b < 32 && ((int64_t)1 << b) < count) ++b;
    return b;
}

}  // namespace

hipError_t launch_bin_sort(ProjPtrs P, BinsPtrs B, void *work, int64_t n, int32_t n_views, int64_t cap,
                           int64_t n_tiles, int tile_w, int tile_h, int32_t *overflow_out, hipStream_t s)
{
    const WorkLayout L = work_layout(n, n_views, cap, n_tiles);
    char *wb = (char *)work;
    uint32_t *keys_a = (uint32_t *)(wb + L.keys_a), *keys_b = (uint32_t *)(wb + L.keys_b);
    uint2 *dvals_a = (uint2 *)(wb + L.dvals_a), *dvals_b = (uint2 *)(wb + L.dvals_b);
    uint32_t *block_sum = (uint32_t *)(wb + L.block_sum), *group_sum = (uint32_t *)(wb + L.group_sum);
    uint32_t *pkeys_a = (uint32_t *)(wb + L.pkeys_a), *pkeys_b = (uint32_t *)(wb + L.pkeys_b);
    uint32_t *pvals_b = (uint32_t *)(wb + L.pvals_b);
    uint32_t *hist = (uint32_t *)(wb + L.hist), *totals = (uint32_t *)(wb + L.totals);
    uint32_t *tkeys_a = (uint32_t *)(wb + L.tkeys_a), *tvals_tmp = (uint32_t *)(wb + L.tvals_a);
    uint32_t *tkeys_b = (uint32_t *)(wb + L.tkeys_b);
    const int64_t R = n * n_views;
    int lw = 0, lh = 0;  // tile sides are powers of two
    while ((1 << lw) < tile_w) ++lw;
    while ((1 << lh) < tile_h) ++lh;
    hipError_t e;

    finalize_counts_kernel<<<1, 64, 0, s>>>(P.hdr, B.hdr, n, n_views, tile_w, tile_h, cap, (uint32_t)n_tiles,
                                            overflow_out);

    // 1. sort the visible records by depth bits, stably in record order: the
    // first pass reads the visibility bits, depth keys and packed tile
    // rectangles in place; each record's rectangle travels with it
    const Count vis_cnt{&B.hdr->n_vis, R};
    bool depth_in_b = false;
    if (R > 0) {
        VisSrc vs;
        vs.bh = B.hdr;
        vs.visbits = P.visbits;
        vs.depth = P.depth;
        vs.n = n;
        vs.vstride = visbits_stride(n);
        vs.nbv = ceil_div(n, kSortTile);
        vs.nbc = n_views * vs.nbv;
        vs.rect = P.rect;
        e = radix_sort(keys_a, dvals_a, keys_b, dvals_b, vis_cnt, 0, 32, hist, totals, s, &depth_in_b, nullptr,
                       &vs);
        if (e != hipSuccess) return e;
    }
    const uint2 *sorted = depth_in_b ? dvals_b : dvals_a;  // (record, packed tile rectangle) in depth order

    // 2. pair offsets in depth order, emit (tile, record) pairs
    // at least one pass, whose scatter records the tile ranges (one tile: a 1-bit pass of zero keys)
    const int tile_bits = bits_for(n_tiles) > 0 ? bits_for(n_tiles) : 1;
    const bool odd = radix_passes(tile_bits) % 2 == 1;
    uint32_t *emit_vals = odd ? pvals_b : B.pair_rec;
    uint32_t *other_vals = odd ? B.pair_rec : pvals_b;
    if (R > 0 && cap > 0) {
        const int64_t nb = ceil_div(R, kCompactTile);
        count_pairs_kernel<<<(unsigned)nb, kSortThreads, 0, s>>>(B.hdr, sorted,
                                                                 (const short4 *)P.bbox, lw, lh, block_sum,
                                                                 group_sum);
        scan_partials_kernel<<<1, 1024, 0, s>>>(block_sum, nb, &B.hdr->n_vis, kCompactTile);
        emit_pairs_kernel<<<(unsigned)ceil_div(R, 256), 256, 0, s>>>(B.hdr, sorted,
                                                                     (const short4 *)P.bbox, P.views, make_div32((uint32_t)n), lw, lh, block_sum,
                                                                     group_sum, pkeys_a, emit_vals);
        // 3. stable sort by global tile id; its last pass records the tile ranges
        if (n_tiles > 0)
            fill_ranges_kernel<<<(unsigned)ceil_div(n_tiles, 256), 256, 0, s>>>(B.tile_range, n_tiles);
        bool pairs_in_b = false;
        const Count pair_cnt{&B.hdr->n_pairs, cap};
        e = radix_sort(pkeys_a, emit_vals, pkeys_b, other_vals, pair_cnt, 0, tile_bits, hist, totals, s,
                       &pairs_in_b, B.tile_range);
        if (e != hipSuccess) return e;
    } else {
        fill_u32_kernel<<<(unsigned)ceil_div(2 * n_tiles, 256), 256, 0, s>>>((uint32_t *)B.tile_range,
                                                                             2 * n_tiles, 0u);
    }
    // 4. work order: heaviest tiles first (one 8-bit pass from the tmp buffers into tile_order)
    if (n_tiles > 0) {
        tile_cost_keys_kernel<<<(unsigned)ceil_div(n_tiles, 256), 256, 0, s>>>(B.tile_range, n_tiles, tkeys_a,
                                                                               tvals_tmp);
        bool in_b = false;
        e = radix_sort(tkeys_a, tvals_tmp, tkeys_b, B.tile_order, Count{nullptr, n_tiles}, 0, 8, hist, totals,
                       s, &in_b);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- allocation-free entry point

// Scratch of dbs_bin_sort_noalloc: one fixed array per GPU, held from the
// library's load until the process ends.  Host code never passes the array's
// name to a kernel (on the host it only names the symbol); it passes the
// device address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[DBS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

hipError_t noalloc_scratch(void **out)
{
    static std::mutex mu;
    static void *per_device[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!per_device[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        per_device[dev] = ptr;
    }
    *out = per_device[dev];
    return hipSuccess;
}

}  // namespace dbs
