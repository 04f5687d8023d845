// Tree construction on gfx950: bounding cube, Morton codes, LDS radix sort, binary radix tree,
// collapsed octree, and the upward pass that forms the pseudo-particles.
//
// Paper: Sec. 3.2 (kernels 1-4 of the GPU Barnes-Hut scheme: bounding box, octree, cell centres and
// moments, sort by location) and Eq. (magCenter) (pseudo-particle = moment sum at the geometric
// centre of the members).  The lock-based insertion of the paper is replaced by the binary radix tree
// construction of T. Karras, "Maximizing parallelism in the construction of BVHs, octrees, and k-d
// trees" (HPG 2012), collapsed to an octree with leaf size leaf_size; the spin-waiting moment kernel
// is replaced by a level-synchronous upward pass (one launch per level, or one workgroup for small trees).
#include "ffbh_internal.h"

namespace ffbh {

// ------------------------------------------------------------------------------------------------
// Bounding cube: lo = componentwise minimum, side = largest extent, scale = 2^21 / side.
// ------------------------------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_bbox_partial(const double *__restrict__ pos, int64_t n,
                                                      double *__restrict__ part,
                                                      uint32_t *__restrict__ status, int enter)
{
    if (enter && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) call_enter(status);
    __shared__ double red[6][256];
    const int b = blockIdx.y;
    const double *p = pos + (int64_t)b * 3 * n;
    double mn[3], mx[3];
    bool bad = false;
    for (int a = 0; a < 3; ++a) { mn[a] = __builtin_inf(); mx[a] = -__builtin_inf(); }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        for (int a = 0; a < 3; ++a) {
            double v = p[a * n + i];
            bad |= !__builtin_isfinite(v);
            if (v < mn[a]) mn[a] = v;
            if (v > mx[a]) mx[a] = v;
        }
    }
    if (bad) set_flag(status, BH_FLAG_NONFINITE);
    for (int a = 0; a < 3; ++a) { red[a][threadIdx.x] = mn[a]; red[3 + a][threadIdx.x] = mx[a]; }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int a = 0; a < 3; ++a) {
                double o = red[a][threadIdx.x + s];
                if (o < red[a][threadIdx.x]) red[a][threadIdx.x] = o;
                o = red[3 + a][threadIdx.x + s];
                if (o > red[3 + a][threadIdx.x]) red[3 + a][threadIdx.x] = o;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[((int64_t)b * kBboxBlocks + blockIdx.x) * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// One workgroup of 256 per system folds the nb partial boxes (min and max are exact in any order).
// Block 0 also clears the level-bucket counters (lvl, 128 words), which the build fills after the octree.
__global__ __launch_bounds__(256) void k_bbox_final(const double *__restrict__ part, int nb,
                                                    double *__restrict__ bbox, uint32_t *__restrict__ lvl,
                                                    double s2_scale)
{
    __shared__ double red[6][256];
    if (blockIdx.x == 0 && threadIdx.x < 128) lvl[threadIdx.x] = 0u;
    const int b = blockIdx.x;
    double v[6];
    for (int a = 0; a < 3; ++a) {
        v[a] = __builtin_inf();
        v[3 + a] = -__builtin_inf();
    }
    for (int k = threadIdx.x; k < nb; k += 256) {
        const double *q = part + ((int64_t)b * kBboxBlocks + k) * 6;
        for (int a = 0; a < 3; ++a) {
            v[a] = fmin(v[a], q[a]);
            v[3 + a] = fmax(v[3 + a], q[3 + a]);
        }
    }
    for (int a = 0; a < 6; ++a) red[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fmin(red[a][threadIdx.x], red[a][threadIdx.x + s]);
                red[3 + a][threadIdx.x] = fmax(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double side = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double e = red[3 + a][0] - red[a][0];
        if (e > side) side = e;
    }
    double *o = bbox + 8 * b;
    o[0] = red[0][0]; o[1] = red[1][0]; o[2] = red[2][0];
    o[3] = side;
    o[4] = side > 0.0 ? 2097152.0 / side : 0.0;
    o[5] = s2_scale;  // factor of the squared cell sides in the node records (node_s2_scale)
}

// ------------------------------------------------------------------------------------------------
// Morton codes: q = min(2^21-1, floor((r - lo) * scale)) per axis, interleaved x-major.
// ------------------------------------------------------------------------------------------------

__device__ inline uint32_t quantise(double r, double lo, double scale)
{
    double t = (r - lo) * scale;
    double f = __builtin_floor(t);
    if (f >= (double)kQMax) return kQMax;
    if (f <= 0.0) return 0u;
    return (uint32_t)f;
}

__global__ __launch_bounds__(256) void k_morton(const double *__restrict__ pos, int64_t n, int64_t ntot,
                                                const double *__restrict__ bbox,
                                                uint64_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= ntot) return;
    int64_t b = o / n, i = o - b * n;
    const double *p = pos + b * 3 * n;
    const double *bb = bbox + 8 * b;
    uint32_t qx = quantise(p[i], bb[0], bb[4]);
    uint32_t qy = quantise(p[n + i], bb[1], bb[4]);
    uint32_t qz = quantise(p[2 * n + i], bb[2], bb[4]);
    keys[o] = morton(qx, qy, qz);
    vals[o] = (uint32_t)o;
}

// ------------------------------------------------------------------------------------------------
// LSD radix sort, 8-bit digits, stable, segmented by system: a tile never straddles two systems, and
// histograms are laid out (system, digit, tile) so one exclusive scan yields every output offset.
// ------------------------------------------------------------------------------------------------

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                             int tiles, int items, int shift,
                                                             uint32_t *__restrict__ hist)
{
    __shared__ uint32_t cnt[kRadixBins];
    const int b = blockIdx.x / tiles, t = blockIdx.x - b * tiles;
    const int64_t tile = (int64_t)kSortThreads * items;
    const int64_t lo = (int64_t)b * n + (int64_t)t * tile;
    const int64_t hi = min(lo + tile, (int64_t)(b + 1) * n);
    cnt[threadIdx.x] = 0;
    // all of this thread's keys are loaded before the first count, so their latencies overlap
    uint32_t d[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = lo + (int64_t)r * kSortThreads + threadIdx.x;
        d[r] = r < items && i < hi ? (uint32_t)(keys[i] >> shift) & (kRadixBins - 1) : kRadixBins;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r)
        if (d[r] < kRadixBins) atomicAdd(&cnt[d[r]], 1u);
    __syncthreads();
    hist[((int64_t)b * kRadixBins + threadIdx.x) * tiles + t] = cnt[threadIdx.x];
}

// Device-wide exclusive scan of a uint32 array in place, in three launches: per-tile sums, a scan of
// the tile sums (one workgroup), and the per-tile scan with its offset.  Tiles are kScanTile entries,
// read and written through LDS so that global accesses are coalesced.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    // inclusive Hillis-Steele over 256 threads in LDS, then shift
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        uint32_t x = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    total = sh[kScanThreads - 1];
    uint32_t r = t ? sh[t - 1] : 0u;
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const uint32_t *__restrict__ a, int64_t len,
                                                             uint32_t *__restrict__ tile_sum)
{
    __shared__ uint32_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < len) s += a[i];
    }
    uint32_t total;
    block_excl_scan(s, sh, total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(uint32_t *__restrict__ tile_sum, int ntiles,
                                                            uint32_t *__restrict__ total_out)
{
    __shared__ uint32_t sh[kScanThreads];
    uint32_t carry = 0;
    for (int base = 0; base < ntiles; base += kScanThreads) {
        const int i = base + (int)threadIdx.x;
        uint32_t v = i < ntiles ? tile_sum[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, sh, tot);
        if (i < ntiles) tile_sum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(uint32_t *__restrict__ a, int64_t len,
                                                             const uint32_t *__restrict__ tile_off)
{
    __shared__ uint32_t tile[kScanTile];
    __shared__ uint32_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int k = 0; k < kScanItems; ++k) {
        const int j = k * kScanThreads + threadIdx.x;
        tile[j] = base + j < len ? a[base + j] : 0u;
    }
    __syncthreads();
    // each thread scans its own run of kScanItems consecutive entries
    uint32_t run = 0;
    for (int k = 0; k < kScanItems; ++k) run += tile[threadIdx.x * kScanItems + k];
    uint32_t total;
    uint32_t off = block_excl_scan(run, sh, total) + tile_off[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        const int j = threadIdx.x * kScanItems + k;
        const uint32_t v = tile[j];
        tile[j] = off;
        off += v;
    }
    __syncthreads();
    for (int k = 0; k < kScanItems; ++k) {
        const int j = k * kScanThreads + threadIdx.x;
        if (base + j < len) a[base + j] = tile[j];
    }
}

// Inclusive scan over the 64 lanes of a wave.
__device__ inline uint32_t wave_incl_scan_u32(uint32_t v, int lane)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t x = __shfl_up(v, off, kWave);
        if (lane >= off) v += x;
    }
    return v;
}

// Exclusive scan of a short array (len <= kScanSmallMax) in one launch of one workgroup: chunks of
// 8192 entries pass through LDS (coalesced loads and stores); each thread scans a run of 8 consecutive
// entries, offset by a wave scan and the wave totals.  LDS index j is padded to j + j/32 against bank
// conflicts of the strided run accesses.
constexpr int kScanSmallThreads = 1024;
constexpr int kScanSmallItems = 8;
constexpr int kScanSmallChunk = kScanSmallThreads * kScanSmallItems;
constexpr int64_t kScanSmallMax = 4 * (int64_t)kScanSmallChunk;

__device__ inline int scan_pad(int j) { return j + (j >> 5); }

__global__ __launch_bounds__(kScanSmallThreads) void k_scan_small(uint32_t *__restrict__ a, int64_t len,
                                                                  uint32_t *__restrict__ total_out)
{
    constexpr int kWaves = kScanSmallThreads / kWave;
    __shared__ uint32_t tile[kScanSmallChunk + kScanSmallChunk / 32];
    __shared__ uint32_t wsum[kWaves];
    const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
    uint32_t carry = 0;
    for (int64_t base = 0; base < len; base += kScanSmallChunk) {
#pragma unroll
        for (int k = 0; k < kScanSmallItems; ++k) {
            const int j = k * kScanSmallThreads + t;
            tile[scan_pad(j)] = base + j < len ? a[base + j] : 0u;
        }
        __syncthreads();
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < kScanSmallItems; ++k) run += tile[scan_pad(t * kScanSmallItems + k)];
        const uint32_t incl = wave_incl_scan_u32(run, lane);
        if (lane == kWave - 1) wsum[wave] = incl;
        __syncthreads();
        uint32_t woff = 0, ctot = 0;
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t x = wsum[w];
            woff += w < wave ? x : 0u;
            ctot += x;
        }
        uint32_t off = carry + woff + incl - run;
#pragma unroll
        for (int k = 0; k < kScanSmallItems; ++k) {
            const int j = scan_pad(t * kScanSmallItems + k);
            const uint32_t v = tile[j];
            tile[j] = off;
            off += v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScanSmallItems; ++k) {
            const int j = k * kScanSmallThreads + t;
            if (base + j < len) a[base + j] = tile[scan_pad(j)];
        }
        carry += ctot;
        __syncthreads();  // tile and wsum are rewritten by the next chunk
    }
    if (t == 0 && total_out) *total_out = carry;
}

// Exclusive scan in place; writes the total to *total if not null.  scratch: one uint32 per tile.
static void scan_excl(uint32_t *a, int64_t len, uint32_t *scratch, uint32_t *total, hipStream_t s)
{
    if (len <= kScanSmallMax) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kScanSmallThreads), 0, s, a, len, total);
        return;
    }
    const int ntiles = (int)((len + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kScanThreads), 0, s, a, len, scratch);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, scratch, ntiles, total);
    hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(kScanThreads), 0, s, a, len, scratch);
}

constexpr int kFusedTiles = 256;

// One pass of the stable LSD sort over one tile of up to kSortThreads * items keys.  Each wave ranks a
// contiguous chunk of 64 * items keys (the keys of equal digit before it in the chunk: match masks from
// ballots plus running per-wave digit counts in LDS); the chunks' counts give every key its position in
// the tile sorted by digit, where the keys are staged in LDS; then each digit's run of the tile is
// written out to consecutive addresses.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, const uint32_t *__restrict__ hist, int64_t n, int tiles, int items, int shift,
    int64_t ntot, int fused)
{
    constexpr int kWaves = kSortThreads / kWave;
    constexpr int kTileMax = kSortThreads * kSortItems;
    __shared__ uint32_t gbase[kRadixBins];        // output offset of the tile's first key of digit d
    __shared__ uint32_t lstart[kRadixBins];       // position of that key in the digit-sorted tile
    __shared__ uint32_t wcnt[kWaves][kRadixBins]; // per-wave digit counts, then per-wave digit offsets
    __shared__ uint32_t dsum[kWaves];
    __shared__ uint64_t skey[kTileMax];
    __shared__ uint32_t sval[kTileMax];
    const int b = blockIdx.x / tiles, t = blockIdx.x - b * tiles;
    const int64_t tile = (int64_t)kSortThreads * items;
    const int64_t lo = (int64_t)b * n + (int64_t)t * tile;
    const int64_t hi = min(lo + tile, (int64_t)(b + 1) * n);
    const int count = (int)(hi - lo);
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const uint32_t dmask = kRadixBins - 1;
    for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0u;

    // this wave's chunk, loaded up front (coalesced, all loads in flight together)
    const int c0 = wave * kWave * items;
    uint64_t key[kSortItems];
    uint32_t val[kSortItems], rank[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int p = c0 + r * kWave + lane;
        const bool valid = r < items && p < count;
        key[r] = valid ? kin[lo + p] : 0ull;
        val[r] = valid ? vin[lo + p] : 0u;
    }
    __syncthreads();  // wcnt cleared
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        if (r < items) {
            const bool valid = c0 + r * kWave + lane < count;
            const uint32_t d = (uint32_t)(key[r] >> shift) & dmask;
            uint64_t m = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < kRadixBits; ++bit) {
                const bool set = (d >> bit) & 1u;
                const uint64_t v = __ballot(set);
                m &= set ? v : ~v;
            }
            const uint32_t before = (uint32_t)__popcll(m & lt);
            // one wave's LDS accesses complete in order: this read sees the previous round's update
            const uint32_t cur = valid ? wcnt[wave][d] : 0u;
            rank[r] = cur + before;
            if (valid && before == 0) wcnt[wave][d] = cur + (uint32_t)__popcll(m);
        }
    }
    __syncthreads();

    // thread tid owns digit tid: per-wave offsets, the tile's digit starts, and the output offset
    uint32_t tot_tile = 0;
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t c = wcnt[w][tid];
        wcnt[w][tid] = tot_tile;
        tot_tile += c;
    }
    {
        const uint32_t incl = wave_incl_scan_u32(tot_tile, lane);
        if (lane == kWave - 1) dsum[wave] = incl;
        __syncthreads();
        uint32_t woff = 0;
        for (int w = 0; w < wave; ++w) woff += dsum[w];
        lstart[tid] = woff + incl - tot_tile;
    }
    if (fused) {
        // hist holds raw counts: the offset of (digit, tile t) is the system's start, plus the keys of
        // smaller digits, plus this digit's keys in earlier tiles
        const uint32_t *hd = hist + ((int64_t)b * kRadixBins + tid) * tiles;
        uint32_t pre = 0, tot = 0;
        if ((tiles & 3) == 0) {
            // rows of a multiple of four counts start 16-byte aligned: read them four at a time, sixteen
            // loads in flight (one at a time, the row's L2 latencies add up to most of the kernel)
            const uint4 *h4 = (const uint4 *)hd;
#pragma unroll 16
            for (int u4 = 0; u4 < tiles / 4; ++u4) {
                const uint4 c = h4[u4];
                const int u = 4 * u4;
                tot += c.x + c.y + c.z + c.w;
                pre += (u < t ? c.x : 0u) + (u + 1 < t ? c.y : 0u) + (u + 2 < t ? c.z : 0u) + (u + 3 < t ? c.w : 0u);
            }
        } else {
#pragma unroll 16
            for (int u = 0; u < tiles; ++u) {
                const uint32_t c = hd[u];
                tot += c;
                pre += u < t ? c : 0u;
            }
        }
        __syncthreads();  // dsum is reused
        const uint32_t incl = wave_incl_scan_u32(tot, lane);
        if (lane == kWave - 1) dsum[wave] = incl;
        __syncthreads();
        uint32_t woff = 0;
        for (int w = 0; w < wave; ++w) woff += dsum[w];
        gbase[tid] = (uint32_t)((int64_t)b * n) + woff + incl - tot + pre;
    } else {
        gbase[tid] = hist[((int64_t)b * kRadixBins + tid) * tiles + t];
    }
    __syncthreads();

    // stage the tile in digit order
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        if (r < items && c0 + r * kWave + lane < count) {
            const uint32_t d = (uint32_t)(key[r] >> shift) & dmask;
            const uint32_t at = lstart[d] + wcnt[wave][d] + rank[r];
            if (at < (uint32_t)kTileMax) {  // always true for a consistent count
                skey[at] = key[r];
                sval[at] = val[r];
            }
        }
    }
    __syncthreads();
    // each digit's run goes to consecutive output addresses
    for (int j = tid; j < count; j += kSortThreads) {
        const uint64_t k = skey[j];
        const uint32_t d = (uint32_t)(k >> shift) & dmask;
        const int64_t at = (int64_t)gbase[d] + (j - (int64_t)lstart[d]);
        if (at >= 0 && at < ntot) {  // always true for a consistent histogram
            kout[at] = k;
            vout[at] = sval[j];
        }
    }
}

// The tiled sort orders the codes by their bits above the low kTieBits only, stably, so particles whose
// codes agree above those bits are left in index order.  With 32 low bits left out the upper bits are the
// cell 2^-10 of the cube wide (and one bit of the next level): at 2^20 particles in the chain workload's
// cube that is 0.17 diameters, a cell no two particles that exclude each other share.  The thread at the
// start of each run of equal upper bits orders the run by the low bits, stably, which gives the order of
// the full codes (ties in index order).  Short runs by insertion; longer ones by a bottom-up merge through
// the second key buffer (free at this point), so any run, even all particles at one point, takes
// O(L log L).
constexpr int kTieInsertMax = 32;

__device__ inline bool low_less(uint64_t a, uint64_t b)
{
    constexpr uint64_t m = (1ull << kTieBits) - 1ull;
    return (a & m) < (b & m);
}

__global__ __launch_bounds__(256) void k_fix_ties(uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                  uint64_t *__restrict__ tkeys, uint32_t *__restrict__ tvals,
                                                  int64_t n, int64_t ntot)
{
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= ntot) return;
    const int64_t b = o / n, end = (b + 1) * n;
    const uint64_t h = keys[o] >> kTieBits;
    if (o > b * n && (keys[o - 1] >> kTieBits) == h) return;  // not the start of a run
    if (o + 1 >= end || (keys[o + 1] >> kTieBits) != h) return;  // a run of one
    int64_t e = o + 2;
    while (e < end && (keys[e] >> kTieBits) == h) ++e;
    const int64_t len = e - o;
    if (len <= kTieInsertMax) {
        for (int64_t i = o + 1; i < e; ++i) {
            const uint64_t k = keys[i];
            const uint32_t v = vals[i];
            int64_t j = i;
            while (j > o && low_less(k, keys[j - 1])) {
                keys[j] = keys[j - 1];
                vals[j] = vals[j - 1];
                --j;
            }
            keys[j] = k;
            vals[j] = v;
        }
        return;
    }
    // bottom-up merge sort of [o, e), stable, ping-ponging between the buffers
    uint64_t *ka = keys, *kb = tkeys;
    uint32_t *va = vals, *vb = tvals;
    for (int64_t w = 1; w < len; w <<= 1) {
        for (int64_t lo = o; lo < e; lo += 2 * w) {
            const int64_t mid = min(lo + w, e), hi = min(lo + 2 * w, e);
            int64_t i = lo, j = mid, k = lo;
            while (i < mid && j < hi) {
                if (low_less(ka[j], ka[i])) { kb[k] = ka[j]; vb[k] = va[j]; ++j; }
                else { kb[k] = ka[i]; vb[k] = va[i]; ++i; }
                ++k;
            }
            while (i < mid) { kb[k] = ka[i]; vb[k] = va[i]; ++i; ++k; }
            while (j < hi) { kb[k] = ka[j]; vb[k] = va[j]; ++j; ++k; }
        }
        uint64_t *kt = ka; ka = kb; kb = kt;
        uint32_t *vt = va; va = vb; vb = vt;
    }
    if (ka != keys)
        for (int64_t i = o; i < e; ++i) {
            keys[i] = ka[i];
            vals[i] = va[i];
        }
}

// Whole sort of one small system in one workgroup (systems of at most kSortSmallMax keys): the keys stay
// in LDS for all eight passes (the full codes, no tie fix needed), so a small system's sort is one launch
// instead of the tiled path's nine (four passes of two launches, then the runs of equal upper bits).
// Each pass is the tile pass of k_radix_scatter over the whole system: every wave ranks a contiguous
// chunk of keys (ballot match masks, running per-wave digit counts), the digit starts and per-wave
// offsets place every key, and the keys move to the other LDS buffer.  Stable, so the result is the
// multi-workgroup sort's.
constexpr int kSortSmallThreads = 512;
constexpr int kSortSmallMax = 2048;

__global__ __launch_bounds__(kSortSmallThreads) void k_sort_small(uint64_t *__restrict__ keys,
                                                                  uint32_t *__restrict__ vals, int n)
{
    constexpr int kWaves = kSortSmallThreads / kWave;
    constexpr int kItems = kSortSmallMax / kSortSmallThreads;  // rounds of 64 keys per wave
    __shared__ uint64_t sk[2][kSortSmallMax];
    __shared__ uint32_t sv[2][kSortSmallMax];
    __shared__ uint32_t wcnt[kWaves][kRadixBins];
    __shared__ uint32_t lstart[kRadixBins];
    __shared__ uint32_t dsum[kRadixBins / kWave];
    const int64_t base = (int64_t)blockIdx.x * n;
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const uint32_t dmask = kRadixBins - 1;
    const int cn = n < kSortSmallMax ? n : kSortSmallMax;
    for (int i = tid; i < cn; i += kSortSmallThreads) {
        sk[0][i] = keys[base + i];
        sv[0][i] = vals[base + i];
    }
    // wave w ranks keys [w * chunk, (w + 1) * chunk) in rounds of 64
    const int chunk = ((cn + kWaves * kWave - 1) / (kWaves * kWave)) * kWave;
    const int c0 = wave * chunk;
    for (int pass = 0; pass < kRadixPasses; ++pass) {
        const int src = pass & 1, dst = src ^ 1, shift = pass * kRadixBits;
        for (int w = 0; w < kWaves; ++w)
            for (int d = tid; d < kRadixBins; d += kSortSmallThreads) wcnt[w][d] = 0u;
        __syncthreads();  // loads (or the previous pass's moves) and the cleared counts are visible
        uint32_t rank[kItems];
        uint32_t dig[kItems];
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const int p = c0 + r * kWave + lane;
            const bool valid = r * kWave < chunk && p < cn;
            const uint32_t d = valid ? (uint32_t)(sk[src][p] >> shift) & dmask : 0u;
            uint64_t m = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < kRadixBits; ++bit) {
                const bool set = (d >> bit) & 1u;
                const uint64_t v = __ballot(set);
                m &= set ? v : ~v;
            }
            const uint32_t before = (uint32_t)__popcll(m & lt);
            // one wave's LDS accesses complete in order: this read sees the previous round's update
            const uint32_t cur = valid ? wcnt[wave][d] : 0u;
            rank[r] = cur + before;
            dig[r] = d;
            if (valid && before == 0) wcnt[wave][d] = cur + (uint32_t)__popcll(m);
        }
        __syncthreads();
        // threads below kRadixBins own one digit: per-wave offsets and the digit's start
        uint32_t tot = 0;
        if (tid < kRadixBins) {
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = wcnt[w][tid];
                wcnt[w][tid] = tot;
                tot += c;
            }
        }
        uint32_t incl = 0;
        if (tid < kRadixBins) {
            incl = wave_incl_scan_u32(tot, lane);
            if (lane == kWave - 1) dsum[wave] = incl;
        }
        __syncthreads();
        if (tid < kRadixBins) {
            uint32_t woff = 0;
            for (int w = 0; w < wave; ++w) woff += dsum[w];
            lstart[tid] = woff + incl - tot;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const int p = c0 + r * kWave + lane;
            if (r * kWave < chunk && p < cn) {
                const uint32_t at = lstart[dig[r]] + wcnt[wave][dig[r]] + rank[r];
                if (at < (uint32_t)kSortSmallMax) {  // always true for consistent counts
                    sk[dst][at] = sk[src][p];
                    sv[dst][at] = sv[src][p];
                }
            }
        }
        __syncthreads();  // every move (and every read of wcnt, lstart) done before the next pass
    }
    // kRadixPasses is even: the sorted keys are in buffer 0
    for (int i = tid; i < cn; i += kSortSmallThreads) {
        keys[base + i] = sk[0][i];
        vals[base + i] = sv[0][i];
    }
}

// Sorted positions (SoA, global over systems).
__global__ __launch_bounds__(256) void k_gather3(const double *__restrict__ src, const uint32_t *__restrict__ perm,
                                                 int64_t n, int64_t ntot, double *__restrict__ dst,
                                                 float *__restrict__ dst32, uint32_t *__restrict__ status)
{
    int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= ntot) return;
    const int64_t o = perm[s];
    if (o >= ntot) {
        set_flag(status, BH_FLAG_TREE);
        return;
    }
    const int64_t b = o / n, i = o - b * n;
    const double *p = src + b * 3 * n;
    bool bad = false;
    for (int a = 0; a < 3; ++a) {
        double v = p[a * n + i];
        bad |= !__builtin_isfinite(v);
        dst[a * ntot + s] = v;
        if (dst32) dst32[a * ntot + s] = (float)v;
    }
    if (bad) set_flag(status, BH_FLAG_NONFINITE);
}

// ------------------------------------------------------------------------------------------------
// Binary radix tree (Karras 2012), one per system over its n sorted codes.  delta(i, j) is the length
// of the common prefix of codes i and j within the 63 code bits; equal codes are told apart by their
// sorted positions (63 + common prefix of the 32-bit positions).  Out-of-range j gives -1.
// ------------------------------------------------------------------------------------------------

__device__ inline int prefix_len(const uint64_t *k, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    uint64_t a = k[i], c = k[j];
    if (a == c) return 63 + __clz((unsigned)(i ^ j));
    return __clzll((long long)(a ^ c)) - 1;
}

__global__ __launch_bounds__(256) void k_karras(const uint64_t *__restrict__ codes, int64_t n, int64_t nint_tot,
                                                int32_t *__restrict__ left, int32_t *__restrict__ right,
                                                int32_t *__restrict__ first, int32_t *__restrict__ last,
                                                int32_t *__restrict__ delta, int32_t *__restrict__ bparent,
                                                int32_t *__restrict__ lparent)
{
    int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= nint_tot) return;
    const int nn = (int)n;
    const int64_t b = g / (n - 1);
    const int i = (int)(g - b * (n - 1));
    const uint64_t *k = codes + b * n;
    const int d = (prefix_len(k, nn, i, i + 1) - prefix_len(k, nn, i, i - 1)) > 0 ? 1 : -1;
    const int dmin = prefix_len(k, nn, i, i - d);
    int lmax = 2;
    while (prefix_len(k, nn, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(k, nn, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = prefix_len(k, nn, i, j);
    int s = 0;
    for (int div = 2;; div <<= 1) {
        const int t = (l + div - 1) / div;
        if (prefix_len(k, nn, i, i + (s + t) * d) > dnode) s += t;
        if (t <= 1) break;
    }
    const int gamma = i + s * d + min(d, 0);
    const int lo = min(i, j), hi = max(i, j);
    const int64_t ib = b * (n - 1), lb = b * n;
    int32_t L, R;
    if (lo == gamma) { L = ~gamma; lparent[lb + gamma] = i; }
    else { L = gamma; bparent[ib + gamma] = i; }
    if (hi == gamma + 1) { R = ~(gamma + 1); lparent[lb + gamma + 1] = i; }
    else { R = gamma + 1; bparent[ib + gamma + 1] = i; }
    left[g] = L;
    right[g] = R;
    first[g] = lo;
    last[g] = hi;
    delta[g] = dnode;
    if (i == 0) bparent[ib] = -1;
}

// ------------------------------------------------------------------------------------------------
// Octree from the binary tree.  A binary node whose members share 3*l but no more code bits has its
// deepest common cell at level lev = min(21, delta / 3).  It starts a new octree cell iff its level
// exceeds its binary parent's; a run of unary cells is stored once, at its deepest level, which
// leaves every pseudo-particle and every acceptance decision unchanged (a unary parent has the same
// members and a larger side).  A cell is in the tree iff its octree parent is internal
// (count > leaf_size and level < 21).  Leaves sit at the top of their run (they are not split).
// ------------------------------------------------------------------------------------------------

__device__ inline int bin_level(const int32_t *delta, int64_t g)
{
    int l = delta[g] / 3;
    return l > kMaxLevel ? kMaxLevel : l;
}

__global__ __launch_bounds__(256) void k_oct_count(int64_t n, int64_t nint_tot, int leaf,
                                                   const int32_t *__restrict__ left,
                                                   const int32_t *__restrict__ right,
                                                   const int32_t *__restrict__ first,
                                                   const int32_t *__restrict__ last,
                                                   const int32_t *__restrict__ delta,
                                                   const int32_t *__restrict__ bparent,
                                                   int32_t *__restrict__ nchild, uint32_t *__restrict__ scan_in,
                                                   uint32_t *__restrict__ status)
{
    int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= nint_tot) return;
    const int64_t b = g / (n - 1), ib = b * (n - 1);
    const int cnt = last[g] - first[g] + 1;
    int out = 0;
    if (cnt <= leaf) {  // no children whether or not the node is in the tree (most nodes)
        nchild[g] = 0;
        scan_in[g] = 0u;
        return;
    }
    const int lev = bin_level(delta, g);
    // is this node the deepest cell of an octree run, and is that cell in the tree?
    const int p = bparent[g];
    bool in_tree;
    if (p < 0) {
        in_tree = true;
    } else if (lev <= bin_level(delta, ib + p)) {
        in_tree = false;  // an intermediate binary split inside one octant digit
    } else {
        // octree parent: nearest binary ancestor that starts a cell (at most 2 binary levels up)
        int x = p;
        for (int up = 0; up < 64; ++up) {
            const int px = bparent[ib + x];
            if (px < 0 || px >= n - 1 || bin_level(delta, ib + x) > bin_level(delta, ib + px)) break;
            x = px;
        }
        const int pc = last[ib + x] - first[ib + x] + 1;
        in_tree = pc > leaf && bin_level(delta, ib + x) < kMaxLevel;
    }
    if (in_tree) {
        if (lev >= kMaxLevel) {
            set_flag(status, BH_FLAG_DEEP_LEAF);
        } else {
            // children: walk the binary subtree down to the nodes that start the next cells
            int32_t stk[8];
            int sp = 0;
            stk[sp++] = right[g];
            stk[sp++] = left[g];
            while (sp > 0) {
                const int32_t c = stk[--sp];
                if (c < 0 || c >= n - 1 || bin_level(delta, ib + c) > lev) {
                    ++out;
                } else if (sp > 5) {  // one octant digit spans at most three binary levels
                    set_flag(status, BH_FLAG_TREE);
                    break;
                } else {
                    stk[sp++] = right[ib + c];
                    stk[sp++] = left[ib + c];
                }
            }
        }
    }
    nchild[g] = out;
    scan_in[g] = (uint32_t)out;
}

// Write the records of the children of every in-tree internal node (and of the roots), and, for each
// leaf among them, its id as the leaf of its members.
__device__ inline void stamp_leaf(int32_t *__restrict__ leaf_of, int64_t first, int count, int64_t end, int32_t id)
{
    for (int k = 0; k < count; ++k)
        if (first + k < end) leaf_of[first + k] = id;
}

__global__ __launch_bounds__(256) void k_oct_emit(int64_t n, int64_t nint_tot, int64_t B, int leaf,
                                                  const int32_t *__restrict__ left,
                                                  const int32_t *__restrict__ right,
                                                  const int32_t *__restrict__ first,
                                                  const int32_t *__restrict__ last,
                                                  const int32_t *__restrict__ delta,
                                                  const int32_t *__restrict__ nchild,
                                                  const uint32_t *__restrict__ scan,
                                                  NodeRec *__restrict__ nodes, int32_t *__restrict__ node_level,
                                                  int32_t *__restrict__ octid, uint32_t *__restrict__ status,
                                                  int64_t max_nodes, int32_t *__restrict__ leaf_of)
{
    int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g == 0) status[2] = (uint32_t)B + (nint_tot > 0 ? status[1] : 0u);  // number of nodes
    // roots: one thread per system (threads g < B); node b is the root of system b
    if (g < B) {
        const int64_t b = g;
        NodeRec r{};
        r.first = (int32_t)(b * n);
        r.count = (int32_t)n;
        r.parent = -1;
        r.child = -1;
        r.nchild = 0;
        int lev = 0;
        if (n > 1 && n > leaf) {
            const int64_t rg = b * (n - 1);
            lev = bin_level(delta, rg);  // deepest cell of the root's run (kMaxLevel: one deep leaf)
            if (nchild[rg] > 0) {
                r.child = (int32_t)(B + scan[rg]);
                r.nchild = nchild[rg];
            }
            octid[rg] = (int32_t)b;
        }
        nodes[b] = r;
        node_level[b] = lev;
        if (r.nchild == 0) stamp_leaf(leaf_of, b * n, (int)n, b * n + n, (int32_t)b);
    }
    if (g >= nint_tot) return;
    const int nc = nchild[g];
    if (nc == 0) return;
    const int64_t b = g / (n - 1), ib = b * (n - 1);
    const int lev = bin_level(delta, g);
    int id = (int)(B + scan[g]);
    if ((int64_t)id + nc > max_nodes) {
        set_flag(status, BH_FLAG_TREE);
        return;
    }
    int32_t stk[8];
    int sp = 0;
    stk[sp++] = right[g];
    stk[sp++] = left[g];
    while (sp > 0) {
        const int32_t c = stk[--sp];
        const bool particle = c < 0;
        if (!particle && c >= n - 1) {
            set_flag(status, BH_FLAG_TREE);
            break;
        }
        if (particle || bin_level(delta, ib + c) > lev) {
            if (id >= B + (int64_t)scan[g] + nc || (particle && ~c >= n)) {
                set_flag(status, BH_FLAG_TREE);
                break;
            }
            NodeRec r{};
            int cf, cc, clev;
            int ch = -1, cn = 0;
            if (particle) {
                cf = ~c; cc = 1; clev = lev + 1;
            } else {
                const int64_t cg = ib + c;
                cf = first[cg];
                cc = last[cg] - first[cg] + 1;
                if (cc > leaf) {
                    clev = bin_level(delta, cg);  // deepest cell of the run; kMaxLevel for a deep leaf
                    if (nchild[cg] > 0) {
                        ch = (int)(B + scan[cg]);
                        cn = nchild[cg];
                    }
                } else {
                    clev = lev + 1;  // a leaf is the first cell of its run
                }
                octid[cg] = id;
            }
            r.first = (int32_t)(b * n + cf);
            r.count = cc;
            r.child = ch;
            r.nchild = cn;
            r.parent = -1;  // set by k_oct_link
            nodes[id] = r;
            node_level[id] = clev;
            if (cn == 0) stamp_leaf(leaf_of, b * n + cf, cc, b * n + n, id);
            ++id;
        } else if (sp > 5) {
            set_flag(status, BH_FLAG_TREE);
            break;
        } else {
            stk[sp++] = right[ib + c];
            stk[sp++] = left[ib + c];
        }
    }
}

// Parent links: every in-tree internal node stamps its id into its children.
__global__ __launch_bounds__(256) void k_oct_link(int64_t nint_tot, int64_t B, const int32_t *__restrict__ nchild,
                                                  const uint32_t *__restrict__ scan,
                                                  const int32_t *__restrict__ octid, NodeRec *__restrict__ nodes,
                                                  int64_t max_nodes)
{
    int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= nint_tot) return;
    const int nc = nchild[g];
    if (nc == 0) return;
    const int self = octid[g];
    const int c0 = (int)(B + scan[g]);
    if (nc < 0 || nc > 8 || (int64_t)c0 + nc > max_nodes) return;
    for (int q = 0; q < nc; ++q) nodes[c0 + q].parent = self;
}

// ------------------------------------------------------------------------------------------------
// Upward pass: first every leaf (in one launch: a leaf sums its members in sorted order starting from
// +0.0, whatever its level), then the internal nodes level by level from the deepest cell level to the
// root (a parent sums its children's sums in octant order, the order they are stored in).  Every child
// of a level-l cell is a leaf or sits at a deeper level, so one launch per level (21 down to 0) sees all
// children finished.  Nodes are bucketed once per build: internal nodes by level (buckets 0..21), leaves
// in bucket kLeafBucket.
//   MODE 0: positions -> centroid S / count and squared side into the node record, and the exact
//           bounding box of the members (used by short-range neighbour queries).
//   MODE 1: moments   -> FP64 moment sum into node_m64 and its FP32 rounding into the record.
// ------------------------------------------------------------------------------------------------

constexpr int kLeafBucket = kMaxLevel + 1;
constexpr int kBuckets = kMaxLevel + 2;

__device__ inline int bucket_of(const NodeRec *__restrict__ nodes, const int32_t *__restrict__ node_level, int64_t i)
{
    const int lev = node_level[i];
    if ((unsigned)lev > (unsigned)kMaxLevel) return -1;
    return nodes[i].nchild == 0 ? kLeafBucket : lev;
}

__global__ __launch_bounds__(256) void k_level_count(const NodeRec *__restrict__ nodes,
                                                     const int32_t *__restrict__ node_level,
                                                     const uint32_t *__restrict__ num_nodes, int64_t max_nodes,
                                                     uint32_t *__restrict__ lvl)
{
    __shared__ uint32_t h[kBuckets];
    if (threadIdx.x < kBuckets) h[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t nn = min((int64_t)*num_nodes, max_nodes);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nn; i += (int64_t)gridDim.x * 256) {
        const int bk = bucket_of(nodes, node_level, i);
        if (bk >= 0) atomicAdd(&h[bk], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kBuckets && h[threadIdx.x]) atomicAdd(&lvl[threadIdx.x], h[threadIdx.x]);
}

// lvl[0..22] counts -> lvl[32..55] bucket starts (exclusive, 24 entries), lvl[64..86] cursors.
__global__ void k_level_starts(uint32_t *lvl)
{
    if (threadIdx.x != 0) return;
    uint32_t acc = 0;
    for (int l = 0; l < kBuckets; ++l) {
        lvl[32 + l] = acc;
        lvl[64 + l] = acc;
        acc += lvl[l];
    }
    lvl[32 + kBuckets] = acc;
}

// One block per 256 node ids: ranks within the block come from LDS atomics, and one global atomic per
// bucket and block reserves the block's slots.
__global__ __launch_bounds__(256) void k_level_scatter(const NodeRec *__restrict__ nodes,
                                                       const int32_t *__restrict__ node_level,
                                                       const uint32_t *__restrict__ num_nodes, int64_t max_nodes,
                                                       uint32_t *__restrict__ lvl, int32_t *__restrict__ lvl_nodes)
{
    __shared__ uint32_t cnt[kBuckets], base[kBuckets];
    const int64_t nn = min((int64_t)*num_nodes, max_nodes);
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if ((int64_t)blockIdx.x * 256 >= nn) return;  // whole block beyond the nodes
    if (threadIdx.x < kBuckets) cnt[threadIdx.x] = 0u;
    __syncthreads();
    const int bk = i < nn ? bucket_of(nodes, node_level, i) : -1;
    const uint32_t r = bk >= 0 ? atomicAdd(&cnt[bk], 1u) : 0u;
    __syncthreads();
    if (threadIdx.x < kBuckets && cnt[threadIdx.x]) base[threadIdx.x] = atomicAdd(&lvl[64 + threadIdx.x], cnt[threadIdx.x]);
    __syncthreads();
    if (bk >= 0 && (int64_t)base[bk] + r < max_nodes) lvl_nodes[base[bk] + r] = (int32_t)i;
}

// MODE 0: member positions -> centroids and s^2; MODE 1: member moments -> FP64 and FP32 moment sums;
// MODE 2: both in one pass (vals = positions, vals2 = moments).  Child sums are read from `sums` (8 doubles
// per node: position sums at 0..2, moment sums at 4..6).
// MODE 0: position sums and centres; 1: moment sums; 2: both; 3: moment sums and first moments
// D = sum_j (r_j - c) m_j^T about the centre c (vals = moments, vals2 = positions; centres from MODE 0/2):
// a leaf sums its members in sorted order, a parent adds its children's D shifted to its own centre,
// D_child + (c_child - c) M_child^T, in octant order.
template <int MODE>
__device__ inline void upward_node(uint32_t q, const double *__restrict__ vals, const double *__restrict__ vals2,
                                   int64_t ntot, int64_t n, NodeRec *__restrict__ nodes, double *__restrict__ sums,
                                   double *__restrict__ node_m64, const int32_t *__restrict__ node_level,
                                   const int32_t *__restrict__ lvl_nodes, const double *__restrict__ bbox,
                                   int64_t max_nodes, double *__restrict__ q64, float *__restrict__ q32)
{
    const int id = lvl_nodes[q];
    if (id < 0 || id >= max_nodes) return;
    const NodeRec nd = nodes[id];
    if (nd.first < 0 || nd.count < 1 || (int64_t)nd.first + nd.count > ntot ||
        (nd.nchild != 0 && (nd.child < 0 || (int64_t)nd.child + nd.nchild > max_nodes)))
        return;
    const int o = MODE == 1 || MODE == 3 ? 4 : 0;  // slot of the (first) sum
    double sx = 0.0, sy = 0.0, sz = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    double D[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (MODE == 3) {
        const double c[3] = {nd.cx, nd.cy, nd.cz};
        if (nd.nchild == 0) {
            for (int k = nd.first; k < nd.first + nd.count; ++k) {
                const double d[3] = {vals2[k] - c[0], vals2[ntot + k] - c[1], vals2[2 * ntot + k] - c[2]};
                const double m[3] = {vals[k], vals[ntot + k], vals[2 * ntot + k]};
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) D[3 * a + b] = D[3 * a + b] + d[a] * m[b];
            }
        } else {
            for (int ch = nd.child; ch < nd.child + nd.nchild; ++ch) {
                const NodeRec cn = nodes[ch];
                const double d[3] = {cn.cx - c[0], cn.cy - c[1], cn.cz - c[2]};
                const double m[3] = {sums[8 * ch + 4], sums[8 * ch + 5], sums[8 * ch + 6]};
                const double *dc = q64 + 16 * (int64_t)ch;
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) D[3 * a + b] = D[3 * a + b] + (dc[3 * a + b] + d[a] * m[b]);
            }
        }
    }
    // sums in member (child) order, as the definition's; unrolled so that several members' loads are in
    // flight at once (the additions stay in order: no reassociation without fast-math)
    if (nd.nchild == 0) {
#pragma unroll 4
        for (int k = nd.first; k < nd.first + nd.count; ++k) {
            sx = sx + vals[k];
            sy = sy + vals[ntot + k];
            sz = sz + vals[2 * ntot + k];
            if (MODE == 2) {
                mx = mx + vals2[k];
                my = my + vals2[ntot + k];
                mz = mz + vals2[2 * ntot + k];
            }
        }
    } else {
#pragma unroll 4
        for (int c = nd.child; c < nd.child + nd.nchild; ++c) {
            sx = sx + sums[8 * c + o];
            sy = sy + sums[8 * c + o + 1];
            sz = sz + sums[8 * c + o + 2];
            if (MODE == 2) {
                mx = mx + sums[8 * c + 4];
                my = my + sums[8 * c + 5];
                mz = mz + sums[8 * c + 6];
            }
        }
    }
    if (MODE == 1 || MODE == 3) {
        mx = sx; my = sy; mz = sz;
    }
    if (MODE == 3) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            q64[16 * (int64_t)id + k] = D[k];
            q32[16 * (int64_t)id + k] = (float)D[k];
        }
    }
    sums[8 * id + o] = sx;
    sums[8 * id + o + 1] = sy;
    sums[8 * id + o + 2] = sz;
    if (MODE == 2) {
        sums[8 * id + 4] = mx;
        sums[8 * id + 5] = my;
        sums[8 * id + 6] = mz;
    }
    if (MODE == 0 || MODE == 2) {
        const double cnt = (double)nd.count;
        nodes[id].cx = sx / cnt;
        nodes[id].cy = sy / cnt;
        nodes[id].cz = sz / cnt;
        const double *bb = bbox + 8 * (nd.first / n);
        const double side = __builtin_ldexp(bb[3], -node_level[id]);
        nodes[id].s2 = side * side * bb[5];  // bb[5]: 1, or 1 / theta^2 for the scaled acceptance test
    }
    if (MODE != 0) {
        node_m64[4 * id] = mx;
        node_m64[4 * id + 1] = my;
        node_m64[4 * id + 2] = mz;
        nodes[id].mx = (float)mx;
        nodes[id].my = (float)my;
        nodes[id].mz = (float)mz;
    }
}

// Level bucket [b0, b1) of the level-sorted node list.
__device__ inline void level_range(const uint32_t *lvl, int level, int64_t max_nodes, uint32_t &b0, uint32_t &b1)
{
    b0 = lvl[32 + level];
    b1 = (int64_t)lvl[32 + level + 1] < max_nodes ? lvl[32 + level + 1] : (uint32_t)max_nodes;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_upward_level(const double *__restrict__ vals,
                                                      const double *__restrict__ vals2, int64_t ntot, int64_t n,
                                                      NodeRec *__restrict__ nodes, double *__restrict__ sums,
                                                      double *__restrict__ node_m64,
                                                      const int32_t *__restrict__ node_level,
                                                      const uint32_t *__restrict__ lvl,
                                                      const int32_t *__restrict__ lvl_nodes,
                                                      const double *__restrict__ bbox, int level,
                                                      int64_t max_nodes, double *__restrict__ q64,
                                                      float *__restrict__ q32)
{
    uint32_t b0, b1;
    level_range(lvl, level, max_nodes, b0, b1);
    for (uint32_t q = b0 + blockIdx.x * 256 + threadIdx.x; q < b1; q += gridDim.x * 256)
        upward_node<MODE>(q, vals, vals2, ntot, n, nodes, sums, node_m64, node_level, lvl_nodes, bbox, max_nodes,
                          q64, q32);
}

// Buckets level_hi down to level_lo in one workgroup (kLeafBucket, the leaves, comes first; then the
// internal nodes of levels 21 .. 0), a barrier between buckets (the children's sums are written by this
// workgroup before their parents read them): where the per-level launches of k_upward_level would cost
// more than the work.  Any number of nodes is handled; few are expected.
constexpr int kUpwardOneThreads = 1024;
constexpr int64_t kUpwardOneMaxNodes = 1 << 16;
// Larger trees: the levels at and below kUpwardDeepLevel hold an internal node only where more than leaf_size
// particles share a cell 2^-kUpwardDeepLevel of the cube wide (none in the dense liquids and chain
// systems simulated), so they take one workgroup launch.  (The top levels are not merged: one
// workgroup walks their few hundred cells more slowly than four grid launches.)
constexpr int kUpwardDeepLevel = 10;

template <int MODE>
__global__ __launch_bounds__(kUpwardOneThreads) void k_upward_all(
    const double *__restrict__ vals, const double *__restrict__ vals2, int64_t ntot, int64_t n,
    NodeRec *__restrict__ nodes, double *__restrict__ sums, double *__restrict__ node_m64,
    const int32_t *__restrict__ node_level, const uint32_t *__restrict__ lvl, const int32_t *__restrict__ lvl_nodes,
    const double *__restrict__ bbox, int64_t max_nodes, double *__restrict__ q64, float *__restrict__ q32,
    int level_hi, int level_lo)
{
    for (int level = level_hi; level >= level_lo; --level) {
        uint32_t b0, b1;
        level_range(lvl, level, max_nodes, b0, b1);
        for (uint32_t q = b0 + threadIdx.x; q < b1; q += kUpwardOneThreads)
            upward_node<MODE>(q, vals, vals2, ntot, n, nodes, sums, node_m64, node_level, lvl_nodes, bbox,
                              max_nodes, q64, q32);
        __syncthreads();
    }
}

template <int MODE>
static void upward(Handle &h, const double *vals, const double *vals2, hipStream_t s)
{
    const Layout &L = h.L;
    Workspace &w = h.w;
    auto one = [&](int level_hi, int level_lo) {
        hipLaunchKernelGGL(k_upward_all<MODE>, dim3(1), dim3(kUpwardOneThreads), 0, s, vals, vals2, L.ntot, L.n,
                           w.nodes, w.node_adj, w.node_m64, w.node_level, w.lvl, w.lvl_nodes, w.bbox, L.max_nodes,
                           w.node_q64, w.node_q32, level_hi, level_lo);
    };
    auto level = [&](int bucket) {
        const unsigned g = grid_for(L.max_nodes, 256, bucket == kLeafBucket ? 1024 : 512);
        hipLaunchKernelGGL(k_upward_level<MODE>, dim3(g), dim3(256), 0, s, vals,
                           vals2, L.ntot, L.n, w.nodes, w.node_adj, w.node_m64, w.node_level, w.lvl, w.lvl_nodes,
                           w.bbox, bucket, L.max_nodes, w.node_q64, w.node_q32);
    };
    if (L.max_nodes <= kUpwardOneMaxNodes) {
        one(kLeafBucket, 0);  // the leaves, then levels 21 .. 0
        return;
    }
    // the leaves hold every member: one launch over all of them; then the internal levels
    level(kLeafBucket);
    one(kMaxLevel, kUpwardDeepLevel);
    for (int l = kUpwardDeepLevel - 1; l >= 0; --l) level(l);
}

// ------------------------------------------------------------------------------------------------
// Host launch sequences
// ------------------------------------------------------------------------------------------------

#define FFBH_TRY(x)                         \
    do {                                    \
        hipError_t e_ = (x);                \
        if (e_ != hipSuccess) return e_;    \
    } while (0)

static void gather_moments(Handle &h, const double *d_mom, hipStream_t s);

hipError_t launch_build(Handle &h, const double *d_pos, hipStream_t s, const double *d_mom, hipStream_t side,
                        bool join, bool enter, const SortedWork &after_sort)
{
    const Layout &L = h.L;
    Workspace &w = h.w;
    const int64_t n = L.n, B = L.B, ntot = L.ntot;
    // partial boxes: at most kBboxBlocks per system, no more than one workgroup per 256 particles
    const int nb = (int)((n + 255) / 256 < kBboxBlocks ? (n + 255) / 256 : kBboxBlocks);
    hipLaunchKernelGGL(k_bbox_partial, dim3((unsigned)nb, (unsigned)B), dim3(256), 0, s, d_pos, n,
                       w.bbox_part, w.status, enter ? 1 : 0);
    hipLaunchKernelGGL(k_bbox_final, dim3((unsigned)B), dim3(256), 0, s, w.bbox_part, nb, w.bbox, w.lvl,
                       node_s2_scale(h.p.theta * h.p.theta));
    hipLaunchKernelGGL(k_morton, dim3(grid_for(ntot, 256)), dim3(256), 0, s, d_pos, n, ntot, w.bbox,
                       w.keys[0], w.vals[0]);
    const int tiles = (int)L.tiles;
    const unsigned sblocks = (unsigned)(B * tiles);
    if (n <= kSortSmallMax) {
        // small systems: the whole sort in LDS, one workgroup per system
        hipLaunchKernelGGL(k_sort_small, dim3((unsigned)B), dim3(kSortSmallThreads), 0, s, w.keys[0], w.vals[0],
                           (int)n);
    } else {
    // the digits above the low kTieBits bits; k_fix_ties then orders the rare runs of equal upper bits
    for (int pass = kTieBits / kRadixBits; pass < kRadixPasses; ++pass) {
        const int src = pass & 1, dst = src ^ 1;
        const int shift = pass * kRadixBits;
        hipLaunchKernelGGL(k_radix_hist, dim3(sblocks), dim3(kSortThreads), 0, s, w.keys[src], n, tiles,
                           L.sort_items, shift, w.hist);
        // up to kFusedTiles tiles per system the scatter derives its offsets from the raw counts
        const int fused = tiles <= kFusedTiles;
        if (!fused) scan_excl(w.hist, (int64_t)L.hist_len, w.scan_tmp, nullptr, s);
        hipLaunchKernelGGL(k_radix_scatter, dim3(sblocks), dim3(kSortThreads), 0, s, w.keys[src],
                           w.vals[src], w.keys[dst], w.vals[dst], w.hist, n, tiles, L.sort_items, shift, ntot,
                           fused);
    }
    hipLaunchKernelGGL(k_fix_ties, dim3(grid_for(ntot, 256)), dim3(256), 0, s, w.keys[0], w.vals[0], w.keys[1],
                       w.vals[1], n, ntot);
    }
    static_assert((kRadixPasses - kTieBits / kRadixBits) % 2 == 0 && kTieBits % kRadixBits == 0,
                  "an even number of tiled passes leaves the sorted data in buffer 0");
    // the sorted data is back in buffer 0
    hipLaunchKernelGGL(k_gather3, dim3(grid_for(ntot, 256)), dim3(256), 0, s, d_pos, w.perm, n, ntot,
                       w.spos, (float *)nullptr, w.status);
    // the sorted codes, permutation and positions and the bounding cube are final from here on
    if (side) {
        hipError_t e = hipEventRecord(h.sorted_ev, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, h.sorted_ev, 0);
        if (e != hipSuccess) return e;
    }
    // Replayed graphs submit the kernels in the order they were captured, so the order of the enqueues
    // below matters: the first octree kernels go first, the side stream's work next (before the rest of
    // the octree, which it runs beside).  With the side stream's work first, the binary radix tree started
    // up to 130 us after the sort in graph replays.
    const int64_t nint = L.bin_int;  // B * (n - 1)
    if (nint > 0) {
        hipLaunchKernelGGL(k_karras, dim3(grid_for(nint, 256)), dim3(256), 0, s, w.codes, n, nint,
                           w.bin_left, w.bin_right, w.bin_first, w.bin_last, w.bin_delta, w.bin_parent,
                           w.leaf_parent);
        hipLaunchKernelGGL(k_oct_count, dim3(grid_for(nint, 256)), dim3(256), 0, s, n, nint,
                           (int)h.p.leaf_size, w.bin_left, w.bin_right, w.bin_first, w.bin_last,
                           w.bin_delta, w.bin_parent, w.bin_nchild, w.bin_scan, w.status);
    }
    if (uses_target_order(L)) launch_target_order(h, side ? side : s);
    if (after_sort) {
        const hipError_t e = after_sort(side ? side : s);
        if (e != hipSuccess) return e;
    }
    if (nint > 0) scan_excl(w.bin_scan, nint, w.scan_tmp, w.status + 1, s);
    hipLaunchKernelGGL(k_oct_emit, dim3(grid_for(nint > B ? nint : B, 256)), dim3(256), 0, s, n, nint, B,
                       (int)h.p.leaf_size, w.bin_left, w.bin_right, w.bin_first, w.bin_last, w.bin_delta,
                       w.bin_nchild, w.bin_scan, w.nodes, w.node_level, w.bin_octid, w.status, L.max_nodes,
                       w.leaf_of);
    if (nint > 0)
        hipLaunchKernelGGL(k_oct_link, dim3(grid_for(nint, 256)), dim3(256), 0, s, nint, B,
                           w.bin_nchild, w.bin_scan, w.bin_octid, w.nodes, L.max_nodes);
    // bucket the nodes by level, then the upward pass for the centroids
    hipLaunchKernelGGL(k_level_count, dim3(grid_for(L.max_nodes, 256, 1024)), dim3(256), 0, s, w.nodes,
                       w.node_level, w.status + 2, L.max_nodes, w.lvl);
    hipLaunchKernelGGL(k_level_starts, dim3(1), dim3(64), 0, s, w.lvl);
    hipLaunchKernelGGL(k_level_scatter, dim3(grid_for(L.max_nodes, 256)), dim3(256), 0, s, w.nodes,
                       w.node_level, w.status + 2, L.max_nodes, w.lvl, w.lvl_nodes);
    if (d_mom) {
        // positions and moments summed in one upward pass
        gather_moments(h, d_mom, s);
        upward<2>(h, w.spos, w.smom, s);
    } else {
        upward<0>(h, w.spos, nullptr, s);
    }
    if (side && join) {
        hipError_t e = hipEventRecord(h.join_ev, side);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, h.join_ev, 0);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// Target order: the traversal takes each wave's targets from a run of consecutive entries of this order.
// Sorted (Morton) order jumps between distant cells at every boundary of the Z curve, and a wave whose
// targets straddle such a jump walks the union of two far-apart neighbourhoods.  The Hilbert curve has no
// jumps (consecutive cells share a face), so waves of targets taken in Hilbert order span smaller regions
// and their union walks visit fewer nodes.  Results depend on the grouping only through the order of
// FP32-mixed partial sums and of the adjoint's reductions.
// ------------------------------------------------------------------------------------------------

// Hilbert index of the cell (x, y, z) of a 2^b grid per axis: Skilling's transform of the axes to the
// transposed index (J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707, 381 (2004)),
// whose bits, interleaved from the most significant down with x first, are the index.
template <int b>
__device__ inline uint32_t hilbert_index(uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t X[3] = {x, y, z};
    // undo the excess work of the curve's reflections and rotations, from the coarsest bit down
#pragma unroll
    for (uint32_t Q = 1u << (b - 1); Q > 1u; Q >>= 1) {
        const uint32_t P = Q - 1u;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const bool invert = (X[i] & Q) != 0u;
            const uint32_t t = invert ? 0u : ((X[0] ^ X[i]) & P);  // exchange the low bits of X[0], X[i]
            X[0] ^= invert ? P : t;
            X[i] ^= t;
        }
    }
    // Gray encode
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0u;
#pragma unroll
    for (uint32_t Q = 1u << (b - 1); Q > 1u; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1u;
    X[0] ^= t; X[1] ^= t; X[2] ^= t;
    return (uint32_t)morton(X[0], X[1], X[2]);
}

// Key of sorted particle o: the Hilbert index of its cell at kHilbertBits bits per axis, read off the top
// bits of its Morton code (the same cube); the value is o itself.
__global__ __launch_bounds__(256) void k_hilbert_keys(const uint64_t *__restrict__ codes, int64_t ntot,
                                                      uint64_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= ntot) return;
    const uint64_t c = codes[o] >> (3 * (kBits - kHilbertBits));
    keys[o] = hilbert_index<kHilbertBits>(compact3(c >> 2), compact3(c >> 1), compact3(c));
    vals[o] = (uint32_t)o;
}

void launch_target_order(Handle &h, hipStream_t s)
{
    const Layout &L = h.L;
    Workspace &w = h.w;
    hipLaunchKernelGGL(k_hilbert_keys, dim3(grid_for(L.ntot, 256)), dim3(256), 0, s, w.codes, L.ntot, w.keys[1],
                       w.vals[1]);
    // three stable 8-bit passes over the 24-bit keys, per system: (keys[1], vals[1]) -> (hkeys, tgt_order)
    // -> (keys[1], vals[1]) -> (hkeys, tgt_order); within a cell the sorted order is kept
    static_assert(kHilbertBits <= kRadixBits, "three radix passes cover the Hilbert keys");
    static_assert(kTargetOrderMin > kSortSmallMax, "systems with a target order take the tiled sort");
    uint64_t *kb[2] = {w.keys[1], w.hkeys};
    uint32_t *vb[2] = {w.vals[1], w.tgt_order};
    const int tiles = (int)L.tiles;
    const unsigned sblocks = (unsigned)(L.B * tiles);
    const int fused = tiles <= kFusedTiles;
    for (int pass = 0; pass < 3; ++pass) {
        const int src = pass & 1, dst = src ^ 1;
        const int shift = pass * kRadixBits;
        hipLaunchKernelGGL(k_radix_hist, dim3(sblocks), dim3(kSortThreads), 0, s, kb[src], L.n, tiles,
                           L.sort_items, shift, w.hist);
        if (!fused) scan_excl(w.hist, (int64_t)L.hist_len, w.hscan_tmp, nullptr, s);
        hipLaunchKernelGGL(k_radix_scatter, dim3(sblocks), dim3(kSortThreads), 0, s, kb[src], vb[src], kb[dst],
                           vb[dst], w.hist, L.n, tiles, L.sort_items, shift, L.ntot, fused);
    }
}

}  // namespace ffbh

namespace ffbh {

// Moments gathered into sorted order (non-finite values flagged) and, in the same pass, the packed source
// record of every sorted particle in the handle's precision (FP64 moment or FP32 moment after the FP64
// position).
__global__ __launch_bounds__(256) void k_gather_pack(const double *__restrict__ mom, const uint32_t *__restrict__ perm,
                                                     const double *__restrict__ spos, int64_t n, int64_t ntot,
                                                     double *__restrict__ smom, double *__restrict__ src64,
                                                     double *__restrict__ src32, uint32_t *__restrict__ status)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= ntot) return;
    const int64_t o = perm[k];
    if (o >= ntot) {
        set_flag(status, BH_FLAG_TREE);
        return;
    }
    const int64_t b = o / n, i = o - b * n;
    const double *p = mom + b * 3 * n;
    const double mx = p[i], my = p[n + i], mz = p[2 * n + i];
    if (!__builtin_isfinite(mx) || !__builtin_isfinite(my) || !__builtin_isfinite(mz))
        set_flag(status, BH_FLAG_NONFINITE);
    smom[k] = mx;
    smom[ntot + k] = my;
    smom[2 * ntot + k] = mz;
    const double x = spos[k], y = spos[ntot + k], z = spos[2 * ntot + k];
    if (src64) {
        double *a = src64 + 6 * k;
        a[0] = x; a[1] = y; a[2] = z; a[3] = mx; a[4] = my; a[5] = mz;
    }
    if (src32) {
        double *r = src32 + 6 * k;
        r[0] = x; r[1] = y; r[2] = z;
        float *f = (float *)(r + 3);
        f[0] = (float)mx; f[1] = (float)my; f[2] = (float)mz; f[3] = 0.0f;
    }
}

// Moments in sorted order and the packed source records of the handle's precision.
static void gather_moments(Handle &h, const double *d_mom, hipStream_t s)
{
    const Layout &L = h.L;
    Workspace &w = h.w;
    const bool mixed = h.p.precision == BH_FP32_MIXED;
    hipLaunchKernelGGL(k_gather_pack, dim3(grid_for(L.ntot, 256)), dim3(256), 0, s, d_mom, w.perm, w.spos, L.n,
                       L.ntot, w.smom, mixed ? (double *)nullptr : (double *)w.src64,
                       mixed ? (double *)w.src32 : (double *)nullptr, w.status);
}

// First moments of every node from the sorted moments and positions already in the workspace (after a
// build with moments): the order-2 cells of an MD step.
hipError_t launch_upward_first_moments(Handle &h, hipStream_t s)
{
    upward<3>(h, h.w.smom, h.w.spos, s);
    return hipGetLastError();
}

hipError_t launch_upward_moments(Handle &h, const double *d_mom, hipStream_t s)
{
    gather_moments(h, d_mom, s);
    if (h.L.expansion == 2)
        upward<3>(h, h.w.smom, h.w.spos, s);
    else
        upward<1>(h, h.w.smom, nullptr, s);
    return hipGetLastError();
}

}  // namespace ffbh
