// Combinatorial track finding on gfx950.
//
//   a1  bin hits per (event, layer, phi bin, z|r bin): count, scan, scatter
//       into 32-byte records (paper Sec. 3.2: hits handed in by the caller;
//       binning makes the per-layer hit search a contiguous range scan);
//   a2  order seeds by (event, eta bin, phi bin), events optionally largest
//       first, with a counting sort, so that a workgroup's seeds share hit
//       bins (paper Sec. 3.2: seeds grouped close in eta and phi for cache
//       reuse of hit data);
//   a3-a7 one persistent kernel walks tiles of seeds through the detector
//       layer by layer (paper Sec. 2: KF-based finding; Sec. 3.1: layer-to-
//       layer propagation; Sec. 4: hit-search windows, candidate scoring):
//       each lane owns one candidate slot (max_cands slots per seed), keeps
//       its state in registers, propagates to its next surface, scans the
//       window's bins for hits passing the chi2 cut, then the seed's slot-0
//       lane merges the children of all its candidates (k-way merge of
//       per-parent sorted lists) and the lanes materialise the survivors with
//       the Kalman update.  Hit lists are recovered from per-step
//       back-pointers at the end.
#include "kf_find.hpp"
#include "kf_math.hpp"
#include "kf_mlp.hpp"

namespace kfmi {

static_assert(sizeof(BinnedHit) == 32, "BinnedHit is two 16-byte loads");
constexpr int kQueues = 8;     // tile queues, one per XCD

// ------------------------------------------------------------------ binning
__device__ inline int phi_bin_of(float phi, int nb)
{
    int b = (int)floorf((phi + float(kPi)) * float(nb) / float(2.0 * kPi));
    return b < 0 ? 0 : (b > nb - 1 ? nb - 1 : b);
}

__device__ inline int coord_bin_of(float v, float lo, float hi, int nb)
{
    float t = floorf((v - lo) * float(nb) / (hi - lo));
    if (!(t >= 0.0f)) t = 0.0f;
    if (t > float(nb - 1)) t = float(nb - 1);
    return (int)t;
}

__device__ inline int event_of(const int32_t* off, int n_events, int64_t i)
{
    int lo = 0, hi = n_events;            // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// exclusive scan over the workgroup of one value per lane; lds holds one int
// per wave
__device__ inline int block_scan_excl(int v, int* total, int* lds)
{
    const int ln = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o);
        if (ln >= o) incl += u;
    }
    if (ln == 63) lds[w] = incl;
    __syncthreads();
    int woff = 0, tot = 0;
    for (int q = 0; q < nw; ++q) {
        const int s = lds[q];
        woff += q < w ? s : 0;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return woff + incl - v;
}

// Hits are binned in two levels of counting sort, all hot counters in LDS:
// (1) group hits by segment = (event, layer): a workgroup histograms a chunk
//     of hits in LDS and reserves each segment's share with one global
//     atomic, then scatters the hit indices;
// (2) one workgroup per segment counts its hits per (phi, z|r) bin in LDS,
//     scans the counts into the segment's bin offsets and writes the 32-byte
//     records contiguously.
constexpr int kSegChunk = 4096;      // hits per workgroup in level 1
constexpr int kSegLocal = 2048;      // segments a level-1 workgroup counts in LDS
constexpr int kChunkEvents = 64;    // events of a chunk whose boundaries level 1 keeps in LDS
constexpr int kScatterBatch = 4;    // hits per lane whose loads the scatter issues together

__device__ inline int event_clamped(const int32_t* off, int n_events, int64_t i)
{
    if (i < off[0]) return 0;
    if (i >= off[n_events]) return n_events - 1;
    return event_of(off, n_events, i);
}

__global__ __launch_bounds__(256) void seg_count_kernel(int64_t n_hits, const int32_t* __restrict__ layer,
                                                        const int32_t* __restrict__ event_off,
                                                        int n_events, int n_layers,
                                                        int32_t* __restrict__ seg_key,
                                                        int32_t* __restrict__ seg_cnt)
{
    __shared__ int h[kSegLocal];
    __shared__ int eoff[kChunkEvents + 2];
    const int64_t c0 = (int64_t)blockIdx.x * kSegChunk;
    const int64_t c1 = c0 + kSegChunk < n_hits ? c0 + kSegChunk : n_hits;
    const int e0 = event_clamped(event_off, n_events, c0);
    const int e1 = event_clamped(event_off, n_events, c1 - 1);
    const int s0 = e0 * n_layers;
    const int ns = (e1 + 1) * n_layers - s0;
    const bool local = ns > 0 && ns <= kSegLocal;   // ns <= 0 only for a decreasing event_off
    // the chunk's event boundaries in LDS: each hit's event by a short search there
    const bool near = e1 >= e0 && e1 - e0 < kChunkEvents;
    if (near)
        for (int k = threadIdx.x; k <= e1 - e0 + 1; k += blockDim.x) eoff[k] = event_off[e0 + k];
    const int64_t all_lo = event_off[0], all_hi = event_off[n_events];
    if (local)
        for (int b = threadIdx.x; b < ns; b += blockDim.x) h[b] = 0;
    __syncthreads();
    for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
        const int l = layer[i];
        int key = -1;
        if (l >= 0 && l < n_layers && i >= all_lo && i < all_hi) {
            int e;
            if (near) {
                int lo = 0, hi = e1 - e0 + 1;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (eoff[mid] <= i) lo = mid;
                    else hi = mid;
                }
                e = e0 + lo;
            } else {
                e = event_of(event_off, n_events, i);
            }
            key = e * n_layers + l;
        }
        seg_key[i] = key;
        if (key >= 0) {
            // (a decreasing event_off could put a hit outside the chunk's
            // event range: such a hit takes the global counter)
            if (local && (unsigned)(key - s0) < (unsigned)ns) atomicAdd(&h[key - s0], 1);
            else atomicAdd(&seg_cnt[key], 1);
        }
    }
    __syncthreads();
    if (local)
        for (int b = threadIdx.x; b < ns; b += blockDim.x)
            if (h[b]) atomicAdd(&seg_cnt[s0 + b], h[b]);
}

__device__ inline int hit_bin(const kf_layer& L, float hx, float hy, float hz)
{
    const int bp = phi_bin_of(atan2f(hy, hx), L.nbin_phi);
    const float v = L.kind == 0 ? hz : sqrtf(hx * hx + hy * hy);
    return bp * L.nbin_2 + coord_bin_of(v, float(L.lo), float(L.hi), L.nbin_2);
}

// Level 1, second pass: each hit's complete record and its bin within the
// layer go to the hit's segment, so that level 2 streams contiguous records
// (the caller's hits may come in any order within an event).
__global__ __launch_bounds__(256) void seg_scatter_kernel(int64_t n_hits, const float* __restrict__ x,
                                                          const float* __restrict__ y,
                                                          const float* __restrict__ z,
                                                          const float* __restrict__ su,
                                                          const float* __restrict__ sv,
                                                          const int32_t* __restrict__ event_off,
                                                          int n_events, const kf_layer* __restrict__ layers,
                                                          int n_layers,
                                                          const int32_t* __restrict__ seg_key,
                                                          const int32_t* __restrict__ seg_off,
                                                          int32_t* __restrict__ seg_fill,
                                                          BinnedHit* __restrict__ seg_rec,
                                                          int32_t* __restrict__ seg_bin)
{
    __shared__ int h[kSegLocal];
    __shared__ int base[kSegLocal];
    __shared__ kf_layer sl[kMaxLayers];
    const int64_t c0 = (int64_t)blockIdx.x * kSegChunk;
    const int64_t c1 = c0 + kSegChunk < n_hits ? c0 + kSegChunk : n_hits;
    const int s0 = event_clamped(event_off, n_events, c0) * n_layers;
    const int ns = (event_clamped(event_off, n_events, c1 - 1) + 1) * n_layers - s0;
    const bool local = ns > 0 && ns <= kSegLocal;   // ns <= 0 only for a decreasing event_off
    for (int l = threadIdx.x; l < n_layers; l += blockDim.x) sl[l] = layers[l];
    if (local) {
        for (int b = threadIdx.x; b < ns; b += blockDim.x) h[b] = 0;
        __syncthreads();
        for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
            const int key = seg_key[i];
            if (key >= 0 && (unsigned)(key - s0) < (unsigned)ns) atomicAdd(&h[key - s0], 1);
        }
        __syncthreads();
        // reserve this chunk's share of every segment it touches
        for (int b = threadIdx.x; b < ns; b += blockDim.x) {
            base[b] = h[b] ? seg_off[s0 + b] + atomicAdd(&seg_fill[s0 + b], h[b]) : 0;
            h[b] = 0;
        }
    }
    __syncthreads();
    // kScatterBatch hits per lane per round: their loads are issued together
    for (int64_t i0 = c0 + threadIdx.x; i0 < c1; i0 += (int64_t)kScatterBatch * blockDim.x) {
        int key[kScatterBatch];
        BinnedHit r[kScatterBatch];
#pragma unroll
        for (int q = 0; q < kScatterBatch; ++q) {
            const int64_t i = i0 + (int64_t)q * blockDim.x;
            key[q] = i < c1 ? seg_key[i] : -1;
            if (key[q] >= 0) {
                r[q].x = x[i];
                r[q].y = y[i];
                r[q].z = z[i];
                r[q].su = su[i];
                r[q].sv = sv[i];
                r[q].idx = (int32_t)i;
            }
        }
#pragma unroll
        for (int q = 0; q < kScatterBatch; ++q) {
            if (key[q] < 0) continue;
            const int k = key[q];
            const int pos = local && (unsigned)(k - s0) < (unsigned)ns
                                ? base[k - s0] + atomicAdd(&h[k - s0], 1)
                                : seg_off[k] + atomicAdd(&seg_fill[k], 1);
            const float rho = sqrtf(r[q].x * r[q].x + r[q].y * r[q].y);
            r[q].cphi = r[q].x / rho;
            r[q].sphi = r[q].y / rho;
            seg_rec[pos] = r[q];
            seg_bin[pos] = hit_bin(sl[k % n_layers], r[q].x, r[q].y, r[q].z);
        }
    }
}

// Level 2: one workgroup per segment sorts its records by bin.  The bin
// counts are histogrammed and scanned in LDS; then every record's place is
// drawn from its bin's counter and, for segments of up to kBinSrcCap records,
// kept as the inverse permutation in LDS, so that the records are written in
// output order (full lines, one read gathered from the segment's own recent
// records each) instead of scattered 32-byte writes that leave their lines
// partly written when the L2 evicts them.  Larger segments scatter directly.
constexpr int kBinThreads = 1024;
constexpr int kBinSrcCap = 12288;
__global__ __launch_bounds__(kBinThreads) void bin_segment_kernel(
    const int32_t* __restrict__ seg_off, const BinnedHit* __restrict__ seg_rec,
    const int32_t* __restrict__ seg_bin, const kf_layer* __restrict__ layers, int n_layers,
    int n_seg, int nb_max, BinLayout bl, int32_t* __restrict__ bin_off, BinnedHit* __restrict__ out)
{
    extern __shared__ int bin_smem[];
    int* hist = bin_smem;                 // [nb_max]
    int* src = bin_smem + nb_max;         // [kBinSrcCap]
    __shared__ int lds[kBinThreads / 64];
    const int seg = blockIdx.x;
    const int e = seg / n_layers, l = seg - e * n_layers;
    const int nb = layers[l].nbin_phi * layers[l].nbin_2;
    const int lo = seg_off[seg], hi = seg_off[seg + 1];
    const int t = threadIdx.x;
    for (int b = t; b < nb; b += kBinThreads) hist[b] = 0;
    __syncthreads();
    for (int i = lo + t; i < hi; i += kBinThreads) atomicAdd(&hist[seg_bin[i]], 1);
    __syncthreads();
    // exclusive scan of the bin counts: lane t takes bins [t*per, (t+1)*per)
    const int per = (nb + kBinThreads - 1) / kBinThreads;
    const int b0 = t * per;
    int s = 0;
    for (int q = 0; q < per; ++q)
        if (b0 + q < nb) s += hist[b0 + q];
    int tot;
    int run = lo + block_scan_excl(s, &tot, lds);
    int32_t* bo = bin_off + (int64_t)e * bl.per_event + bl.base[l];
    for (int q = 0; q < per; ++q)
        if (b0 + q < nb) {
            const int c = hist[b0 + q];
            hist[b0 + q] = run;
            bo[b0 + q] = run;
            run += c;
        }
    if (seg == n_seg - 1 && t == 0) bin_off[(int64_t)(e + 1) * bl.per_event] = hi;
    __syncthreads();
    if (hi - lo <= kBinSrcCap) {
        for (int i = lo + t; i < hi; i += kBinThreads) src[atomicAdd(&hist[seg_bin[i]], 1) - lo] = i;
        __syncthreads();
        for (int j = t; j < hi - lo; j += kBinThreads) out[lo + j] = seg_rec[src[j]];
    } else {
        for (int i = lo + t; i < hi; i += kBinThreads) out[atomicAdd(&hist[seg_bin[i]], 1)] = seg_rec[i];
    }
}

// ------------------------------------------------------------------ prefix sums
// Exclusive prefix sum of n int32 in three launches (no library scan, so that
// the pass contains kernels only and can be captured into a graph): per-chunk
// totals, an in-place scan of the totals by one workgroup, and a rescan of
// each chunk from its offset.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;

__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const int32_t* __restrict__ in,
                                                                   int64_t n,
                                                                   int32_t* __restrict__ bsum)
{
    __shared__ int lds[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x;
    int s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t i = base + (int64_t)q * kScanThreads;
        s += i < n ? in[i] : 0;
    }
    int tot;
    (void)block_scan_excl(s, &tot, lds);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void scan_top_kernel(int32_t* __restrict__ bsum, int nb)
{
    __shared__ int lds[1024 / 64];
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int i = b0 + (int)threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        int tot;
        const int ex = block_scan_excl(v, &tot, lds);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const int32_t* __restrict__ in,
                                                                  int64_t n,
                                                                  const int32_t* __restrict__ bsum,
                                                                  int32_t* __restrict__ out)
{
    __shared__ int lds[kScanThreads / 64];
    // lane t takes kScanItems consecutive values of the chunk
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = base + q < n ? in[base + q] : 0;
        s += v[q];
    }
    int tot;
    int run = bsum[blockIdx.x] + block_scan_excl(s, &tot, lds);
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
}

// ------------------------------------------------------------------ seed order
constexpr int kSeedCells = 64 * 64;   // eta x phi cells per event
constexpr int kRankMaxEvents = 16384; // events ranked by size for the largest-first order

// Position of each event in the processing order: by hit count, largest
// first, ties by event index (a permutation of 0..n_events-1).
__global__ __launch_bounds__(256) void event_rank_kernel(const int32_t* __restrict__ event_off,
                                                         int n_events, int32_t* __restrict__ erank)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_events) return;
    const int ne = event_off[e + 1] - event_off[e];
    int r = 0;
    for (int q = 0; q < n_events; ++q) {
        const int nq = event_off[q + 1] - event_off[q];
        r += (nq > ne || (nq == ne && q < e)) ? 1 : 0;
    }
    erank[e] = r;
}

__global__ __launch_bounds__(256) void seed_cell_kernel(int64_t n, int64_t ld, const float* __restrict__ par,
                                                        const int32_t* __restrict__ seed_event,
                                                        int n_events,
                                                        const int32_t* __restrict__ erank,
                                                        int32_t* __restrict__ cnt,
                                                        int32_t* __restrict__ cell)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float th = par[5 * ld + i], ph = par[4 * ld + i];
    int e = seed_event[i];
    e = e < 0 ? 0 : (e >= n_events ? n_events - 1 : e);
    if (erank) e = erank[e];
    // eta over [-3, 3) and phi over [-pi, pi) in 64 bins each; a non-finite
    // angle falls into bin 0
    const float eta = -logf(tanf(0.5f * th));
    float fe = floorf((eta + 3.0f) * (64.0f / 6.0f));
    fe = fe >= 0.0f ? (fe < 63.0f ? fe : 63.0f) : 0.0f;
    float fp = floorf((ph + float(kPi)) * (64.0f / float(2.0 * kPi)));
    fp = fp >= 0.0f ? (fp < 63.0f ? fp : 63.0f) : 0.0f;
    const int c = e * kSeedCells + (int)fe * 64 + (int)fp;
    atomicAdd(&cnt[c], 1);
    cell[i] = c;
}

__global__ __launch_bounds__(256) void seed_scatter_kernel(int64_t n, const int32_t* __restrict__ cell,
                                                           const int32_t* __restrict__ off,
                                                           int32_t* __restrict__ cnt,
                                                           int32_t* __restrict__ order)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell[i];
    order[off[c] + atomicSub(&cnt[c], 1) - 1] = (int32_t)i;
}

// The scatter leaves a cell's seeds in arbitrary order; sort each cell by
// seed index so that tiles are the same from run to run.  Cells above
// kCellSortMax seeds (only degenerate inputs pile up so) keep the scatter order.
constexpr int kCellSortMax = 256;
__global__ __launch_bounds__(256) void cell_sort_kernel(int64_t n_cells, const int32_t* __restrict__ off,
                                                        int32_t* __restrict__ order)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int lo = off[c], hi = off[c + 1];
    if (hi - lo < 2 || hi - lo > kCellSortMax) return;
    for (int i = lo + 1; i < hi; ++i) {
        const int32_t v = order[i];
        int j = i - 1;
        while (j >= lo && order[j] > v) {
            order[j + 1] = order[j];
            --j;
        }
        order[j + 1] = v;
    }
}

// Tiles of seeds of like cost.  A tile runs as long as its slowest seed,
// and low-pT seeds in the central barrel (loopers, which curl back through
// the layers with ever wider windows) walk longest, so inside each tile
// queue's contiguous range of the processing order the seeds are
// partitioned, stably, by a cost class of |q/pT| and |eta|, costliest first:
// fewer tiles wait on one looper, and the long tiles start first instead of
// ending the pass.  The costliest class, the central loopers, comes in tiles
// of half the seeds: a tile's window scan is shared by its candidates, so
// such a tile ends in about half the time, and the few longest tiles no
// longer outlast the rest of the pass.
constexpr int kCostClasses = 4;

// seeds in a tile of the costliest class: half a tile
__host__ __device__ inline int looper_tile_seeds(int S)
{
    return S / 2 > 1 ? S / 2 : 1;
}
__device__ inline int cost_class(float c, float theta)
{
    // |theta - pi/2| < 0.4803: |eta| < 0.5; < 0.8658: |eta| < 1
    const float a = fabsf(c), e = fabsf(theta - 1.57079633f);
    if (a > 1.0f / 0.6f && e < 0.4803f) return 0;   // central loopers, pT < 0.6 GeV
    if (a > 1.0f / 0.7f && e < 0.8658f) return 1;   // pT < 0.7 GeV, |eta| < 1
    return a > 1.0f ? 2 : 3;                         // pT < 1 GeV, the rest
}

// Two passes over blocks of kCostBlock entries of each queue range [q chunk,
// (q + 1) chunk) of the cell order (chunk is a whole number of tiles): the
// blocks' class counts, then each block places its entries at the class's
// base in the range plus the class's entries in earlier blocks, lanes and
// waves (a stable partition).
constexpr int kCostBlock = 1024;

__device__ inline void cost_block_range(int64_t n, int64_t chunk, int nbq, int64_t* lo, int64_t* hi)
{
    const int q = blockIdx.x / nbq, b = blockIdx.x - q * nbq;
    const int64_t qhi = (int64_t)(q + 1) * chunk < n ? (int64_t)(q + 1) * chunk : n;
    *lo = (int64_t)q * chunk + (int64_t)b * kCostBlock;
    *hi = *lo + kCostBlock < qhi ? *lo + kCostBlock : qhi;
}

__global__ __launch_bounds__(kCostBlock) void cost_count_kernel(int64_t n, int64_t ld,
                                                                const float* __restrict__ par,
                                                                const int32_t* __restrict__ order,
                                                                int64_t chunk, int nbq,
                                                                int32_t* __restrict__ cnt)
{
    __shared__ int tot[kCostClasses];
    int64_t lo, hi;
    cost_block_range(n, chunk, nbq, &lo, &hi);
    const int t = threadIdx.x;
    if (t < kCostClasses) tot[t] = 0;
    __syncthreads();
    const int64_t i = lo + t;
    const int k = i < hi ? cost_class(par[3 * ld + order[i]], par[5 * ld + order[i]]) : -1;
    for (int c = 0; c < kCostClasses; ++c) {
        const unsigned long long m = __ballot(k == c);
        if ((t & 63) == 0 && m) atomicAdd(&tot[c], __popcll(m));
    }
    __syncthreads();
    if (t < kCostClasses) cnt[(size_t)blockIdx.x * kCostClasses + t] = tot[t];
}

__global__ __launch_bounds__(kCostBlock) void cost_place_kernel(int64_t n, int64_t ld,
                                                                const float* __restrict__ par,
                                                                const int32_t* __restrict__ order,
                                                                int64_t chunk, int nbq,
                                                                const int32_t* __restrict__ cnt,
                                                                int32_t* __restrict__ out,
                                                                int32_t* __restrict__ queue_loopers)
{
    __shared__ int wtot[kCostBlock / 64][kCostClasses];   // per wave and class
    __shared__ int base[kCostClasses];                      // class base of this block in the range
    int64_t lo, hi;
    cost_block_range(n, chunk, nbq, &lo, &hi);
    const int q = blockIdx.x / nbq, b = blockIdx.x - q * nbq;
    const int t = threadIdx.x, wave = t >> 6, ln = t & 63;
    if (b == 0 && t == 0) {
        // the range's costliest-class seeds (its head after the partition)
        int c0 = 0;
        for (int bb = 0; bb < nbq; ++bb) c0 += cnt[((size_t)q * nbq + bb) * kCostClasses];
        queue_loopers[q] = c0;
    }
    if (lo >= hi) return;
    if (t < kCostClasses) {
        // entries of the range in the costlier classes, then this class's in earlier blocks
        int before = 0, costlier = 0;
        for (int bb = 0; bb < nbq; ++bb) {
            const int32_t* c = cnt + ((size_t)q * nbq + bb) * kCostClasses;
            for (int k = 0; k < t; ++k) costlier += c[k];
            if (bb < b) before += c[t];
        }
        base[t] = costlier + before;
    }
    const int64_t i = lo + t;
    const int k = i < hi ? cost_class(par[3 * ld + order[i]], par[5 * ld + order[i]]) : -1;
    int below = 0;
    for (int c = 0; c < kCostClasses; ++c) {
        const unsigned long long m = __ballot(k == c);
        if (ln == 0) wtot[wave][c] = __popcll(m);
        if (k == c)
            below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    }
    __syncthreads();
    if (k >= 0) {
        int pos = base[k] + below;
        for (int w = 0; w < wave; ++w) pos += wtot[w][k];
        out[(int64_t)q * chunk + pos] = order[i];
    }
}

// ------------------------------------------------------------------ find
// LDS writes of one wave made visible to that wave's other lanes
__device__ inline void wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A hit's place in a candidate's child list, (chi2, hit index) ascending, as
// one unsigned key: the float's bits made monotone (-0 taken as +0) above
// the non-negative index.
__device__ inline uint64_t child_key(float c2, int32_t id)
{
    uint32_t u = __float_as_uint(c2);
    if (u == 0x80000000u) u = 0u;
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((uint64_t)u << 32) | (uint32_t)id;
}

__device__ inline float child_key_chi2(uint64_t key)
{
    const uint32_t u = (uint32_t)(key >> 32);
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

// A child's place in its seed's selection: more hits first, then lower chi2
// (as child_key's bits), then parent slot j and child c.
__device__ inline uint64_t merge_key(int nhits, float c2, int j, int c)
{
    uint32_t u = __float_as_uint(c2);
    if (u == 0x80000000u) u = 0u;
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    const uint32_t nh = nhits < 0 ? 0u : nhits > 255 ? 255u : (uint32_t)nhits;
    return ((uint64_t)(255u - nh) << 56) | ((uint64_t)u << 24) | ((uint64_t)j << 16) |
           ((uint64_t)c << 8);
}

// Row stride of the window owners' position covariance in LDS: six values
// padded to whole 16-byte reads (three for FP64, two for FP32)
template <typename C> constexpr int kOwnCov = sizeof(C) == 8 ? 6 : 8;

template <typename C>
__device__ inline void load_owner_cov(const C* r, C pc[6])
{
    if constexpr (sizeof(C) == 8) {
        const double2 a = *(const double2*)r, b = *(const double2*)(r + 2), c = *(const double2*)(r + 4);
        pc[0] = a.x; pc[1] = a.y; pc[2] = b.x; pc[3] = b.y; pc[4] = c.x; pc[5] = c.y;
    } else {
        const float4 a = *(const float4*)r;
        const float2 b = *(const float2*)(r + 4);
        pc[0] = a.x; pc[1] = a.y; pc[2] = a.z; pc[3] = a.w; pc[4] = b.x; pc[5] = b.y;
    }
}

// LDS layout of one workgroup (W lanes); arrays lane-minor unless noted
template <typename C>
struct FindShared {
    C* ocov;            // [W][kOwnCov] window owner's predicted position covariance
                        //          P00 P01 P02 P11 P12 P22 (16-byte rows)
    float* pchi2;       // [W]      chi2 of each lane's candidate
    int32_t* meta;      // [4][W]   nhits, misses, status, (done | (layer + 1) << 8)
    float* cchi2;       // [kMaxCands][W]  accepted hit chi2, ascending
    int32_t* cbidx;     // [kMaxCands][W]  binned index of those hits
    int32_t* nchild;    // [W]
    int8_t* sel;        // [S][kMaxCands][2]  (parent slot, child index)
    int32_t* nsel;      // [S]
    kf_layer* layers;   // [n_layers]
    NavOrder* nav;      // surface orders of the dynamic navigation
    int32_t* misc;      // [4] the tile: first position in the order, seed count
    // cooperative window scan, per lane (owner of a window) and per wave
    float* orec;        // [W][8] window owner record: predicted x, y, z, cos and sin of its
                        //        azimuth, sin(dphi), wv, flags (two 16-byte reads)
    int32_t* seg;       // [n_waves][3][kSeg] queued phi rows: owner lane, first hit, count
    int32_t* segpre;    // [n_waves][kSeg + 1] prefix of the rows' hit counts
    int32_t* acc;       // [n_waves][3][kAcc] per owner lane its accepted hits' first and last
                        // entry ([0, 64), [64, 128)); the entries' hit index; their binned index
    float* accc2;       // [n_waves][kAcc] their chi2
    int32_t* rowp;      // [n_waves][5][64] per owner lane: row prefix, first row, bins, base, sizes
};

constexpr int kSeg = 128;       // phi rows queued per wave per round
constexpr int kScanBatch = 4;   // hits per lane in flight in the scan
constexpr int kAcc = 64 * kScanBatch;
constexpr int kInsBatch = 4;    // accepted hits an owner loads together

__host__ __device__ inline size_t find_shared_bytes(int W, int S, int nl, size_t csize)
{
    size_t b = 0;
    b += csize * (csize == 8 ? 6 : 8) * W;
    b += sizeof(float) * W;
    b += sizeof(int32_t) * 4 * W;
    b += sizeof(float) * kMaxCands * W;
    b += sizeof(int32_t) * kMaxCands * W;
    b += sizeof(int32_t) * W;
    b += sizeof(int32_t) * S;
    b = (b + 15) & ~size_t(15);
    b += sizeof(kf_layer) * nl;
    b += sizeof(NavOrder);
    b += sizeof(int32_t) * 4;
    b += 2 * S * kMaxCands;
    b = (b + 15) & ~size_t(15);
    const size_t nw = (W + 63) / 64;
    b += sizeof(float) * 8 * W;
    b += sizeof(int32_t) * nw * (3 * kSeg + kSeg + 1 + 3 * kAcc);
    b += sizeof(float) * nw * kAcc;
    b += sizeof(int32_t) * nw * 5 * 64;
    return (b + 15) & ~size_t(15);
}

// waves per SIMD the register allocation is held to (a build-time tuning knob)
#ifndef KF_FIND_WAVES
#define KF_FIND_WAVES 2
#endif

template <typename T, typename C, typename U, bool LEARN, bool MAT, bool STEER, bool FIELD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KF_FIND_WAVES))) void find_kernel(
    FindArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int W = blockDim.x;
    const int S = a.seeds_per_tile;
    const int MC = a.prm.max_cands;
    const int nl = a.n_layers;
    // seeds and outputs are stored in T; in registers a candidate's state is
    // held in T and its covariance in C (the update runs in U)
    const T* scov = (const T*)a.scov;
    T* ocov = (T*)a.ocov;
    FindShared<C> sh;
    {
        unsigned char* q = smem;
        sh.ocov = (C*)q;
        q += sizeof(C) * kOwnCov<C> * W;
        sh.pchi2 = (float*)q;
        q += sizeof(float) * W;
        sh.meta = (int32_t*)q;
        q += sizeof(int32_t) * 4 * W;
        sh.cchi2 = (float*)q;
        q += sizeof(float) * kMaxCands * W;
        sh.cbidx = (int32_t*)q;
        q += sizeof(int32_t) * kMaxCands * W;
        sh.nchild = (int32_t*)q;
        q += sizeof(int32_t) * W;
        sh.nsel = (int32_t*)q;
        q += sizeof(int32_t) * S;
        q = smem + (((size_t)(q - smem) + 15) & ~size_t(15));
        sh.layers = (kf_layer*)q;
        q += sizeof(kf_layer) * nl;
        sh.nav = (NavOrder*)q;
        q += sizeof(NavOrder);
        sh.misc = (int32_t*)q;
        q += sizeof(int32_t) * 4;
        sh.sel = (int8_t*)q;
        q += 2 * S * kMaxCands;
        q = smem + (((size_t)(q - smem) + 15) & ~size_t(15));
        const int nw = (W + 63) / 64;
        sh.orec = (float*)q;
        q += sizeof(float) * 8 * W;
        sh.seg = (int32_t*)q;
        q += sizeof(int32_t) * nw * 3 * kSeg;
        sh.segpre = (int32_t*)q;
        q += sizeof(int32_t) * nw * (kSeg + 1);
        sh.acc = (int32_t*)q;
        q += sizeof(int32_t) * nw * 3 * kAcc;
        sh.accc2 = (float*)q;
        q += sizeof(float) * nw * kAcc;
        sh.rowp = (int32_t*)q;
    }
    const int t = threadIdx.x;
    for (int l = t; l < nl; l += W) sh.layers[l] = a.layers[l];
    if (t == 0) build_nav_order(a.layers, nl, sh.nav);   // read after the tile loop's barrier
    // seeds never straddle waves: wave w holds seeds w*SPW .. w*SPW + SPW - 1
    const int SPW = seeds_per_wave(W, MC);
    const int ln64 = t & 63;
    const int s_loc = (t >> 6) * SPW + ln64 / MC;
    const int slot = ln64 % MC;
    const bool lane_ok = ln64 / MC < SPW && s_loc < S;
    const int lbase = t - slot;             // lane of this seed's slot 0
    const T kb = T(kKappa) * T(a.prm.bz);
    const float cut = float(a.prm.chi2_cut);
    unsigned n_prop = 0, n_upd = 0, n_chi2 = 0, n_kept = 0;   // per lane: far below 2^32
    int n_newton = 0, n_disk = 0, n_guess = 0, n_fallback = 0;
    int2* bp_base = a.bp + (size_t)blockIdx.x * nl * S * kMaxCands;

    for (;;) {
        __syncthreads();
        if (t == 0) {
            // the processing order is split into kQueues contiguous ranges of
            // whole tiles, one per XCD (workgroups are dispatched to the XCDs
            // round-robin), so that a range's neighbouring eta-phi tiles share
            // that XCD's L2; a workgroup whose range is exhausted takes tiles
            // from the others.  A range's costliest-class seeds, at its head,
            // come in tiles of SL seeds, the rest in tiles of S.
            const int64_t cs = (int64_t)((a.n_tiles + kQueues - 1) / kQueues) * S;
            const int SL = looper_tile_seeds(S);
            const int home = blockIdx.x % kQueues;
            int start = -1, cnt = 0;
            for (int d = 0; d < kQueues; ++d) {
                const int q = (home + d) % kQueues;
                const int64_t lo = q * cs;
                const int64_t hi = lo + cs < a.n_seeds ? lo + cs : a.n_seeds;
                if (lo >= hi) continue;
                const int nq = (int)(hi - lo);
                int c0 = a.queue_loopers[q];
                c0 = c0 < 0 ? 0 : (c0 > nq ? nq : c0);
                const int nlt = (c0 + SL - 1) / SL;
                const int i = atomicAdd(&a.tile_counter[q], 1);
                if (i < nlt) {
                    start = (int)lo + i * SL;
                    cnt = c0 - i * SL < SL ? c0 - i * SL : SL;
                    break;
                }
                const int64_t j0 = c0 + (int64_t)(i - nlt) * S;   // first seed of a full tile
                if (j0 < nq) {
                    start = (int)(lo + j0);
                    cnt = nq - j0 < S ? (int)(nq - j0) : S;
                    break;
                }
            }
            sh.misc[0] = start;
            sh.misc[1] = cnt;
        }
        __syncthreads();
        const int tstart = sh.misc[0], tcount = sh.misc[1];
        if (tstart < 0) break;

        const bool valid = lane_ok && s_loc < tcount;
        const int sid = valid ? a.order[tstart + s_loc] : 0;
        int ev = valid ? a.seed_event[sid] : 0;
        const bool bad_event = ev < 0 || ev >= a.n_events;
        if (bad_event) ev = 0;
        // candidate registers
        T p[6];
        C P[21];
        float chi2 = 0.0f;
        int nhits = 0, misses = 0;
        uint32_t status = 0;
        bool occupied = valid && slot == 0;
        bool done = true;
        if (occupied) {
#pragma unroll
            for (int k = 0; k < 6; ++k) p[k] = T(a.spar[k * a.sld + sid]);
#pragma unroll
            for (int k = 0; k < 21; ++k) P[k] = C(scov[k * a.sld + sid]);
            chi2 = a.schi2[sid];
            nhits = (a.sndf[sid] + 5) / 2;
            status = a.sstatus[sid] | (bad_event ? (uint32_t)KF_ST_BADINPUT : 0u);
            done = (status & kFreezeMask) != 0;
        } else {
#pragma unroll
            for (int k = 0; k < 6; ++k) p[k] = T(0);
#pragma unroll
            for (int k = 0; k < 21; ++k) P[k] = C(0);
        }
        // steering: the seed's region and the plan entry after its last seed
        // layer (every lane of the seed computes the same)
        int rg = 0, pos = 0;
        if constexpr (STEER) {
            if (valid) {
                const double eta = -log(tan(0.5 * (double)a.spar[5 * a.sld + sid]));
                rg = -1;
                for (int g = 0; g < a.steer->n; ++g)
                    if (eta >= a.steer->eta_lo[g] && eta < a.steer->eta_hi[g]) {
                        rg = g;
                        break;
                    }
                int start = -1;
                if (rg >= 0) {
                    for (int q = 0; q < 3; ++q) {
                        const int hi = a.seed_hits[q * a.sld + sid];
                        if (hi < 0 || hi >= a.n_hits) continue;
                        const int hl = a.hit_layer[hi];
                        for (int j = 0; j < a.steer->len[rg]; ++j)
                            if (a.steer->layers[rg][j] == hl && j + 1 > start) start = j + 1;
                    }
                }
                if (start < 0) {
                    if (occupied && !done) {
                        status |= KF_ST_UNREACHABLE;
                        done = true;
                    }
                    rg = 0;
                    start = 0;
                }
                pos = start;
            }
        }
        int nsteps = 0;
        for (int step = 0; step < nl; ++step) {
            const bool live = occupied && !done;
            if (!__syncthreads_or(live)) break;
            // ---- a3: navigate and propagate (LEARN: the whole wave first
            // evaluates the learned start of its candidates' barrel solves)
            T s_guess = T(-1);
            if (LEARN) {
                float f[kMlpIn] = {0, 0, 0, 0, 0, 0, 0, 0};
                const int bl = live ? next_barrel(p, sh.layers, *sh.nav) : -1;
                if (bl >= 0) mlp_features(p, sh.layers[bl], a.prm, f);
                const float y = mlp_wave(a.mlp, f);
                if (bl >= 0) {
                    s_guess = T(mlp_guess(f, y));
                    ++n_guess;
                }
            }
            int pl = -1;
            if (live) {
                T s;
                int layer;
                T fl = T(0);
                T fq[6];
                if constexpr (FIELD && STEER)
                    layer = steer_next_field(p, sh.layers, a.steer->layers[rg], a.steer->len[rg], &pos,
                                             a.prm, &fl, fq, &status, &n_newton, &n_disk);
                else if constexpr (FIELD)
                    layer = navigate_field(p, sh.layers, nl, a.prm, &fl, fq, &status, &n_newton,
                                           &n_disk, s_guess >= T(0) ? s_guess / Tr<T>::sin_(p[5]) : T(-1),
                                           LEARN ? a.prm.mlp_max_iter : 0, &n_fallback);
                else if constexpr (STEER)
                    layer = steer_next(p, sh.layers, a.steer->layers[rg], a.steer->len[rg], &pos,
                                       a.prm, kb, &s, &status, &n_newton, &n_disk);
                else
                    layer = navigate(p, sh.layers, *sh.nav, a.prm, kb, &s, &status, &n_newton, &n_disk,
                                     s_guess, LEARN ? a.prm.mlp_max_iter : 0, &n_fallback);
                if (layer < 0) {
                    done = true;
                } else {
                    ++n_prop;
                    const kf_layer L = sh.layers[layer];
                    if constexpr (FIELD)
                        field_transport(p, P, fq, fl, a.prm, L.kind, T(L.r_or_z));
                    else
                        transport(p, P, s, kb, L.kind, T(L.r_or_z));
                    if (a.material) {
                        if constexpr (MAT)
                            add_material(p, P, L, a.mat, T(a.prm.mass));
                        else
                            add_scatter(p, P, L.kind, T(L.x0), T(a.prm.mass));
                    }
                    bool fin = true;
#pragma unroll
                    for (int k = 0; k < 6; ++k) fin &= isfinite(p[k]);
                    if (fin) {
                        pl = layer;
                    } else {
                        status |= KF_ST_NAN;
                        done = true;
                    }
                }
            }
            // ---- a4: hit-search window, then the window's bins scanned by the
            // whole wave together.  Per-candidate windows differ widely (a diffuse
            // state can cover many rows of bins), so lanes queue their rows and
            // the wave walks the flattened (row, hit) list 64 x kScanBatch hits at
            // a time; accepted hits are compacted with a ballot and each owner
            // lane inserts its own into its sorted list.
            if (lane_ok) {
#pragma unroll
                for (int k = 0; k < 3; ++k) sh.orec[t * 8 + k] = float(p[k]);
                sh.pchi2[t] = chi2;
                C* oc = sh.ocov + t * kOwnCov<C>;
                oc[0] = P[pk(0, 0)];
                oc[1] = P[pk(0, 1)];
                oc[2] = P[pk(0, 2)];
                oc[3] = P[pk(1, 1)];
                oc[4] = P[pk(1, 2)];
                oc[5] = P[pk(2, 2)];
            }
            // this candidate's accepted hits, best first: key and binned index
            uint64_t lk[kMaxCands];
            int32_t lbi[kMaxCands];
#pragma unroll
            for (int k = 0; k < kMaxCands; ++k) {
                lk[k] = ~0ull;
                lbi[k] = -1;
            }
            int nacc = 0;
            int nrow = 0, row_lo = 0, v0 = 0, v1 = 0, np = 1, n2 = 1, row0 = 0;
            if (pl >= 0) {
                const kf_layer L = sh.layers[pl];
                const Window<T> Wn = make_window<T, C>(p, P, L, T(cut));
                if (Wn.ok) {
                    np = L.nbin_phi;
                    n2 = L.nbin_2;
                    int b_lo = 0, b_hi = np - 1;
                    if (!Wn.all_phi) {
                        const T phi = Tr<T>::atan2_(p[1], p[0]);
                        b_lo = (int)Tr<T>::floor_((phi - Wn.dphi + T(kPi)) * T(np) / T(2.0 * kPi));
                        b_hi = (int)Tr<T>::floor_((phi + Wn.dphi + T(kPi)) * T(np) / T(2.0 * kPi));
                        if (b_hi - b_lo + 1 >= np || b_hi < b_lo) {
                            b_lo = 0;
                            b_hi = np - 1;
                        }
                    }
                    nrow = b_hi - b_lo + 1;
                    row_lo = b_lo;
                    v0 = coord_bin_of(float(Wn.vlo), float(L.lo), float(L.hi), n2);
                    v1 = coord_bin_of(float(Wn.vhi), float(L.lo), float(L.hi), n2);
                    row0 = ev * a.bl.per_event + a.bl.base[pl];
                    const T rho = Tr<T>::sqrt_(p[0] * p[0] + p[1] * p[1]);
                    sh.orec[t * 8 + 3] = float(p[0] / rho);
                    sh.orec[t * 8 + 4] = float(p[1] / rho);
                    sh.orec[t * 8 + 5] = float(Wn.sin_dphi);
                    sh.orec[t * 8 + 6] = float(Wn.wv);
                    sh.orec[t * 8 + 7] = __int_as_float((Wn.all_phi ? 1 : 0) | (L.kind << 1));
                }
            }
            {
                const int wave = t >> 6, ln = t & 63;
                const int wlanes = (W - (wave << 6)) < 64 ? (W - (wave << 6)) : 64;
                int32_t* sg_own = sh.seg + wave * 3 * kSeg;
                int32_t* sg_h0 = sg_own + kSeg;
                int32_t* sg_len = sg_h0 + kSeg;
                int32_t* sg_pre = sh.segpre + wave * (kSeg + 1);
                // accepted hits are compacted in hit order, and the flattened hits
                // run owner by owner, so each owner's accepted hits of a round form
                // one range [ac_first, ac_last]
                int32_t* ac_first = sh.acc + wave * 3 * kAcc;
                int32_t* ac_last = ac_first + 64;
                int32_t* ac_id = ac_first + kAcc;
                int32_t* ac_bi = ac_id + kAcc;
                float* ac_c2 = sh.accc2 + wave * kAcc;
                // wave-wide exclusive prefix sum (and total) of one int per lane
                auto wave_scan = [&](int v, int* total) {
                    int incl = v;
                    for (int o = 1; o < 64; o <<= 1) {
                        const int u = __shfl_up(incl, o);
                        if (ln >= o) incl += u;
                    }
                    *total = __shfl(incl, wlanes - 1);
                    return incl - v;
                };
                // rows of every lane, flattened: lane o owns rows [rowpre[o],
                // rowpre[o] + nrow_o) of the wave's row list
                ac_first[ln] = 0x7fffffff;
                ac_last[ln] = -1;
                int R = 0;
                const int rpre = wave_scan(nrow, &R);
                // the row parameters of each owner, for the lanes that expand its rows
                int32_t* rw_par = sh.rowp + wave * 5 * 64;
                rw_par[ln] = rpre;
                rw_par[64 + ln] = row_lo;
                rw_par[128 + ln] = v0 | (v1 << 16);
                rw_par[192 + ln] = row0;
                rw_par[256 + ln] = np | (n2 << 16);
                wave_fence();
                const int segcap = 2 * wlanes < kSeg ? 2 * wlanes : kSeg;
                for (int rr0 = 0; rr0 < R; rr0 += segcap) {
                    // (1) queue rows rr0 .. rr0 + segcap - 1, two per lane; their bin
                    //     ranges are loaded together
                    const int nseg = R - rr0 < segcap ? R - rr0 : segcap;
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        const int j = r * wlanes + ln;
                        if (j < nseg) {
                            const int g = rr0 + j;
                            int lo = 0, hi = wlanes;      // rowpre[lo] <= g < rowpre[hi]
                            while (hi - lo > 1) {
                                const int mid = (lo + hi) >> 1;
                                if (rw_par[mid] <= g) lo = mid;
                                else hi = mid;
                            }
                            const int o = lo;
                            const int bb = rw_par[64 + o] + (g - rw_par[o]);
                            const int vv = rw_par[128 + o], pp = rw_par[256 + o];
                            const int onp = pp & 0xFFFF, on2 = pp >> 16;
                            const int rb = rw_par[192 + o] + (((bb % onp) + onp) % onp) * on2;
                            const int h0 = a.bin_off[rb + (vv & 0xFFFF)];
                            const int h1 = a.bin_off[rb + (vv >> 16) + 1];
                            sg_own[j] = o;
                            sg_h0[j] = h0;
                            sg_len[j] = h1 - h0;
                        }
                    }
                    wave_fence();
                    // (2) prefix of the queued rows' hit counts, two rows per lane
                    const int la = 2 * ln < nseg ? sg_len[2 * ln] : 0;
                    const int lb = 2 * ln + 1 < nseg ? sg_len[2 * ln + 1] : 0;
                    int H = 0;
                    const int pre = wave_scan(la + lb, &H);
                    if (2 * ln < nseg) sg_pre[2 * ln] = pre;
                    if (2 * ln + 1 < nseg) sg_pre[2 * ln + 1] = pre + la;
                    if (ln == 0) sg_pre[nseg] = H;
                    wave_fence();
                    // (3) the flattened hits, 64 x kScanBatch per round.  Lane ln
                    //     walks its own contiguous segment of the list, kScanBatch
                    //     hits per round, so that a round holds hits of many owners
                    //     and their insertions below run side by side.  Owners
                    //     still rise with the lane, so a round's accepted hits of
                    //     one owner stay one range of the compaction.
                    const int nround = (H + wlanes * kScanBatch - 1) / (wlanes * kScanBatch);
                    const int gseg = ln * kScanBatch * nround;   // first hit of the segment
                    // the lane's current row, held in registers: its end in the
                    // list, owner, and binned index minus list position
                    int row = 0, r_end = H, r_own = -1, r_base = 0;
                    if (gseg < H) {
                        int hi = nseg;                            // sg_pre[row] <= gseg < sg_pre[hi]
                        while (hi - row > 1) {
                            const int mid = (row + hi) >> 1;
                            if (sg_pre[mid] <= gseg) row = mid;
                            else hi = mid;
                        }
                        r_end = sg_pre[row + 1];
                        r_own = sg_own[row];
                        r_base = sg_h0[row] - sg_pre[row];
                    }
                    for (int ir = 0; ir < nround; ++ir) {
                        float4 r0[kScanBatch], r1[kScanBatch];
                        int own[kScanBatch], bix[kScanBatch];
                        const int gb = gseg + ir * kScanBatch;
#pragma unroll
                        for (int q = 0; q < kScanBatch; ++q) {
                            const int g = gb + q;
                            own[q] = -1;
                            bix[q] = 0;
                            if (g < H) {
                                while (g >= r_end) {                 // sg_pre[nseg] = H > g
                                    ++row;
                                    r_end = sg_pre[row + 1];
                                    r_own = sg_own[row];
                                    r_base = sg_h0[row] - sg_pre[row];
                                }
                                own[q] = r_own;
                                bix[q] = r_base + g;
                            }
                            r0[q] = *(const float4*)&a.bh[bix[q]].x;
                            r1[q] = *(const float4*)&a.bh[bix[q]].sv;
                        }
                        bool okq[kScanBatch];
                        float c2q[kScanBatch];
#pragma unroll
                        for (int q = 0; q < kScanBatch; ++q) {
                            bool ok = false;
                            float c2f = 0.0f;
                            const int o = own[q];
                            if (o >= 0) {
                                const int ot = (wave << 6) + o;
                                const float hcp = r1[q].y, hsp = r1[q].z;
                                const float4 oa = *(const float4*)&sh.orec[ot * 8];
                                const float4 ob = *(const float4*)&sh.orec[ot * 8 + 4];
                                const T ox = T(oa.x), oy = T(oa.y), oz = T(oa.z);
                                const T cpp = T(oa.w), spp = T(ob.x);
                                const T sin_dphi = T(ob.y), wv = T(ob.z);
                                const int fl = __float_as_int(ob.w);
                                const int kind = fl >> 1;
                                // |azimuth difference| <= dphi (< pi/2): same half-plane, |sin| bounded
                                bool pass = (fl & 1) || (T(hcp) * cpp + T(hsp) * spp > T(0) &&
                                                         !(Tr<T>::abs_(T(hsp) * cpp - T(hcp) * spp) >
                                                           sin_dphi));
                                if (pass) {
                                    const T rv = kind == 0 ? T(r0[q].z) - oz
                                                           : T(hcp) * (T(r0[q].x) - ox) +
                                                                 T(hsp) * (T(r0[q].y) - oy);
                                    pass = !(Tr<T>::abs_(rv) > wv);
                                }
                                if (pass) {
                                    HitFrame<U> f;
                                    f.hx = U(r0[q].x);
                                    f.hy = U(r0[q].y);
                                    f.hz = U(r0[q].z);
                                    f.c = U(hcp);
                                    f.s = U(hsp);
                                    f.vu = U(r0[q].w) * U(r0[q].w);
                                    f.vv = U(r1[q].x) * U(r1[q].x);
                                    C pc[6];
                                    load_owner_cov(sh.ocov + ot * kOwnCov<C>, pc);
                                    const U c2u = hit_chi2_pos<U>(U(ox), U(oy), U(oz), U(pc[0]), U(pc[1]),
                                                                  U(pc[2]), U(pc[3]), U(pc[4]), U(pc[5]),
                                                                  f, kind);
                                    ++n_chi2;
                                    ok = c2u < U(cut);
                                    c2f = float(c2u);
                                }
                            }
                            okq[q] = ok;
                            c2q[q] = c2f;
                        }
                        // compaction in hit order (lane-major: a lane's hits are
                        // consecutive), each entry widening its owner's range
                        int nok = 0;
#pragma unroll
                        for (int q = 0; q < kScanBatch; ++q) nok += okq[q] ? 1 : 0;
                        // exclusive prefix of nok (< 8) over the lanes, bit by bit
                        static_assert(kScanBatch < 8, "nok takes three bits");
                        int pos = 0;
#pragma unroll
                        for (int b = 0; b < 3; ++b) {
                            const uint64_t m = __ballot((nok >> b) & 1);
                            pos += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))
                                   << b;
                        }
#pragma unroll
                        for (int q = 0; q < kScanBatch; ++q)
                            if (okq[q]) {
                                ac_id[pos] = __float_as_int(r1[q].w);
                                ac_bi[pos] = bix[q];
                                ac_c2[pos] = c2q[q];
                                atomicMin(&ac_first[own[q]], pos);
                                atomicMax(&ac_last[own[q]], pos);
                                ++pos;
                            }
                        wave_fence();
                        // (4) owners take their accepted hits; one that cannot enter
                        // the sorted list (not below its last entry) is only counted
                        const int j1 = ac_last[ln];
                        for (int jb = ac_first[ln]; jb <= j1; jb += kInsBatch) {
                            // the batch's entries are loaded together
                            float cb[kInsBatch];
                            int32_t ib[kInsBatch], bb[kInsBatch];
#pragma unroll
                            for (int u = 0; u < kInsBatch; ++u) {
                                const int j = jb + u <= j1 ? jb + u : j1;
                                cb[u] = ac_c2[j];
                                ib[u] = ac_id[j];
                                bb[u] = ac_bi[j];
                            }
#pragma unroll
                            for (int u = 0; u < kInsBatch; ++u) {
                                if (jb + u > j1) break;
                                uint64_t e = child_key(cb[u], ib[u]);
                                int32_t bi = bb[u];
                                ++nacc;
                                if (!(e < lk[kMaxCands - 1])) continue;
                                // the list is ascending, so "e below entry q" holds
                                // from the insertion point on: every slot takes
                                // its own, its predecessor's or the new entry,
                                // all decided from the old entries at once
                                bool lt[kMaxCands];
#pragma unroll
                                for (int q = 0; q < kMaxCands; ++q) lt[q] = e < lk[q];
#pragma unroll
                                for (int q = kMaxCands - 1; q > 0; --q) {
                                    lk[q] = lt[q] ? (lt[q - 1] ? lk[q - 1] : e) : lk[q];
                                    lbi[q] = lt[q] ? (lt[q - 1] ? lbi[q - 1] : bi) : lbi[q];
                                }
                                lk[0] = lt[0] ? e : lk[0];
                                lbi[0] = lt[0] ? bi : lbi[0];
                            }
                        }
                        ac_first[ln] = 0x7fffffff;
                        ac_last[ln] = -1;
                        wave_fence();
                    }
                    // the queue is rewritten next round: every lane is done reading it
                    wave_fence();
                }
            }
            // ---- publish this lane's step outcome and children
            if (lane_ok) {
                sh.meta[0 * W + t] = nhits;
                sh.meta[1 * W + t] = misses;
                sh.meta[2 * W + t] = (int32_t)status;
                sh.meta[3 * W + t] = (done ? 1 : 0) | ((pl + 1) << 8) | (pos << 16);
                const int nk = nacc < MC ? nacc : MC;
                sh.nchild[t] = occupied ? nk : -1;
#pragma unroll
                for (int k = 0; k < kMaxCands; ++k) {
                    sh.cchi2[k * W + t] = lk[k] == ~0ull ? 3.0e38f : child_key_chi2(lk[k]);
                    sh.cbidx[k * W + t] = lbi[k];
                }
            }
            __syncthreads();
            // ---- a5: per-seed selection (k-way merge of per-parent sorted children)
            // by the seed's slot-0 lane, the parents' list heads held in
            // registers: one LDS read per pick after the initial loads
            if (valid && slot == 0) {
                const int base = lbase;
                // list heads as merge keys; parents fill slots 0, 1, ...: the
                // first empty slot ends them
                uint64_t K[kMaxCands];
                bool stop = false;
#pragma unroll
                for (int j = 0; j < kMaxCands; ++j) {
                    const int nkj = j < MC ? sh.nchild[base + j] : -1;
                    stop = stop || nkj < 0;
                    K[j] = ~0ull;
                    if (!stop) {
                        // head: the best child (nk == 0: the child without a hit)
                        const int nh = sh.meta[0 * W + base + j];
                        const float c0 = sh.pchi2[base + j];
                        K[j] = nkj > 0 ? merge_key(nh + 1, c0 + sh.cchi2[0 * W + base + j], j, 0)
                                       : merge_key(nh, c0, j, 0);
                    }
                }
                int nsel = 0;
                for (int r = 0; r < MC; ++r) {
                    uint64_t best = K[0];
#pragma unroll
                    for (int j = 1; j < kMaxCands; ++j) best = K[j] < best ? K[j] : best;
                    if (best == ~0ull) break;
                    const int bj = (int)(best >> 16) & 0xFF, c = (int)(best >> 8) & 0xFF;
                    sh.sel[(s_loc * kMaxCands + r) * 2 + 0] = (int8_t)bj;
                    sh.sel[(s_loc * kMaxCands + r) * 2 + 1] = (int8_t)c;
                    ++nsel;
                    // advance the winner's list: its next hit child, then the
                    // child without a hit, then nothing
                    const int tj = base + bj, cn = c + 1;
                    const int n = sh.nchild[tj], h0 = sh.meta[0 * W + tj];
                    const float cc0 = sh.pchi2[tj];
                    const float cx = sh.cchi2[(cn < kMaxCands ? cn : kMaxCands - 1) * W + tj];
                    const uint64_t nkey = cn < n    ? merge_key(h0 + 1, cc0 + cx, bj, cn)
                                          : cn == n ? merge_key(h0, cc0, bj, cn)
                                                    : ~0ull;
#pragma unroll
                    for (int j = 0; j < kMaxCands; ++j) K[j] = j == bj ? nkey : K[j];
                }
                sh.nsel[s_loc] = nsel;
            }
            __syncthreads();
            // ---- a6: materialise the surviving children (Kalman update for hit
            // children).  A child copies its parent's predicted state from the
            // parent's registers (same wave); every lane takes part in the copy.
            int sel_j = 0, sel_c = 0, src = ln64;
            bool occ_new = false;
            if (valid) {
                occ_new = slot < sh.nsel[s_loc];
                if (occ_new) {
                    sel_j = sh.sel[(s_loc * kMaxCands + slot) * 2 + 0];
                    sel_c = sh.sel[(s_loc * kMaxCands + slot) * 2 + 1];
                    src = (lbase + sel_j) & 63;
                }
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) p[k] = __shfl(p[k], src);
#pragma unroll
            for (int k = 0; k < 21; ++k) P[k] = __shfl(P[k], src);
            if (valid) {
                occupied = occ_new;
                int2 bpe = make_int2(-1, 0xFF00);
                if (occupied) {
                    const int j = sel_j;
                    const int c = sel_c;
                    const int tj = lbase + j;
                    chi2 = sh.pchi2[tj];
                    nhits = sh.meta[0 * W + tj];
                    misses = sh.meta[1 * W + tj];
                    status = (uint32_t)sh.meta[2 * W + tj];
                    const int m3 = sh.meta[3 * W + tj];
                    done = (m3 & 1) != 0;
                    const int ppl = ((m3 >> 8) & 0xFF) - 1;
                    if constexpr (STEER) pos = (m3 >> 16) & 0xFF;
                    const int nk = sh.nchild[tj];
                    if (ppl >= 0) {
                        ++n_kept;
                        if (c < nk) {
                            const int bi = sh.cbidx[c * W + tj];
                            const BinnedHit hh = a.bh[bi];
                            HitFrame<U> f;
                            f.hx = U(hh.x);
                            f.hy = U(hh.y);
                            f.hz = U(hh.z);
                            f.c = U(hh.cphi);
                            f.s = U(hh.sphi);
                            f.vu = U(hh.su) * U(hh.su);
                            f.vv = U(hh.sv) * U(hh.sv);
                            U c2 = U(0);
                            const int r = kf_update<T, C, U>(p, P, f, sh.layers[ppl].kind, &c2);
                            ++n_upd;
                            if (r) {
                                status |= (uint32_t)r;
                                done = true;
                            }
                            chi2 = chi2 + sh.cchi2[c * W + tj];
                            nhits += 1;
                            misses = 0;
                            bpe = make_int2(hh.idx, j | (ppl << 8));
                        } else {
                            misses += 1;
                            if (misses > a.prm.max_miss) done = true;
                            bpe = make_int2(-1, j | (ppl << 8));
                        }
                    } else {
                        bpe = make_int2(-1, j | 0xFF00);
                    }
                    bp_base[((size_t)step * S + s_loc) * kMaxCands + slot] = bpe;
                }
            }
            ++nsteps;
        }
        // ---- a7: best candidate (slot 0, candidates are kept sorted) and its hit list
        if (valid && slot == 0) {
            const int64_t ol = a.n_layers;
            int32_t* oh = a.out_hits + (int64_t)sid * ol;
            // a layer visited more than once (a looper curling back) reports its
            // latest hit: walk the back-pointers from the last step and keep the
            // first hit met per layer, then the seed hits where nothing came later
            for (int l = 0; l < nl; ++l) oh[l] = -1;
            int k = 0;
            for (int st = nsteps - 1; st >= 0; --st) {
                const int2 e = bp_base[((size_t)st * S + s_loc) * kMaxCands + k];
                const int lay = (e.y >> 8) & 0xFF;
                if (e.x >= 0 && lay < nl && oh[lay] < 0) oh[lay] = e.x;
                k = e.y & 0xFF;
            }
            for (int q = 2; q >= 0; --q) {
                const int hi = a.seed_hits[q * a.sld + sid];
                if (hi >= 0 && hi < a.n_hits) {
                    const int hl = a.hit_layer[hi];
                    if (hl >= 0 && hl < nl && oh[hl] < 0) oh[hl] = hi;
                }
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) a.opar[q * a.old + sid] = float(p[q]);
#pragma unroll
            for (int q = 0; q < 21; ++q) ocov[q * a.old + sid] = T(P[q]);
            a.ochi2[sid] = chi2;
            a.ondf[sid] = 2 * nhits - 5;
            a.ostatus[sid] = status;
        }
    }
    if (a.counters) {
        // wave-level reduction of the per-lane counts, one atomic per wave
        unsigned long long c[kFindCounters] = {(unsigned long long)n_prop, (unsigned long long)n_upd,
                                               (unsigned long long)n_chi2, (unsigned long long)n_newton,
                                               (unsigned long long)n_disk, (unsigned long long)n_guess,
                                               (unsigned long long)n_fallback, (unsigned long long)n_kept};
#pragma unroll
        for (int q = 0; q < kFindCounters; ++q) {
            for (int o = 32; o > 0; o >>= 1) c[q] += __shfl_xor(c[q], o);
            if ((t & 63) == 0) atomicAdd(&a.counters[q], c[q]);
        }
    }
}

// ------------------------------------------------------------------ host side
namespace {
inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
}

size_t find_shared_size(int W, int S, int nl, int prec)
{
    return find_shared_bytes(W, S, nl, prec == KF_PREC_FP32 ? sizeof(float) : sizeof(double));
}

// Instantiations: (precision) x (plain, learned, steered; each also in the
// parametrised field) x (material map); learned and steered exclude each other.
template <typename T, typename C, typename U, bool LEARN, bool MAT>
static hipError_t find_occ2(bool steer, bool field, int W, size_t lds, int* out)
{
    if (field) {
        if constexpr (!LEARN)
            if (steer)
                return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    out, find_kernel<T, C, U, false, MAT, true, true>, W, lds);
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, find_kernel<T, C, U, LEARN, MAT, false, true>,
                                                            W, lds);
    }
    if constexpr (!LEARN)
        if (steer)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                out, find_kernel<T, C, U, false, MAT, true, false>, W, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, find_kernel<T, C, U, LEARN, MAT, false, false>,
                                                        W, lds);
}

template <typename T, typename C, typename U, bool LEARN>
static hipError_t find_occ(bool mat, bool steer, bool field, int W, size_t lds, int* out)
{
    return mat ? find_occ2<T, C, U, LEARN, true>(steer, field, W, lds, out)
               : find_occ2<T, C, U, LEARN, false>(steer, field, W, lds, out);
}

hipError_t find_max_blocks_per_cu(int W, int S, int nl, int prec, bool learn, bool mat, bool steer,
                                  bool field, int* out)
{
    const size_t lds = find_shared_size(W, S, nl, prec);
    if (prec == KF_PREC_FP32)
        return learn ? find_occ<float, float, float, true>(mat, steer, field, W, lds, out)
                     : find_occ<float, float, float, false>(mat, steer, field, W, lds, out);
    return learn ? find_occ<float, double, double, true>(mat, steer, field, W, lds, out)
                 : find_occ<float, double, double, false>(mat, steer, field, W, lds, out);
}

hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    unsigned g = blocks_for(n, 256);
    if (g > 4096) g = 4096;
    fill_i32_kernel<<<g, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* bsum, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const unsigned nb = blocks_for(n, kScanChunk);
    scan_reduce_kernel<<<nb, kScanThreads, 0, s>>>(in, n, bsum);
    scan_top_kernel<<<1, 1024, 0, s>>>(bsum, (int)nb);
    scan_apply_kernel<<<nb, kScanThreads, 0, s>>>(in, n, bsum, out);
    return hipGetLastError();
}

hipError_t launch_bin(const FindPlan& pl, const kf_hits* h, const int32_t* event_off, int n_events,
                      const kf_layer* d_layers, int n_layers, hipStream_t s)
{
    hipError_t e;
    const int64_t n_seg = (int64_t)n_events * n_layers;
    if ((e = launch_fill(pl.seg_cnt, 2 * (n_seg + 1), 0, s)) != hipSuccess) return e;   // cnt and fill
    const unsigned nchunk = blocks_for(h->n, kSegChunk);
    if (h->n > 0) {
        seg_count_kernel<<<nchunk, 256, 0, s>>>(h->n, h->layer, event_off, n_events, n_layers,
                                                pl.hit_key, pl.seg_cnt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = launch_scan(pl.seg_cnt, pl.seg_off, n_seg + 1, pl.bsum, s)) != hipSuccess) return e;
    if (h->n > 0) {
        seg_scatter_kernel<<<nchunk, 256, 0, s>>>(h->n, h->x, h->y, h->z, h->su, h->sv, event_off,
                                                  n_events, d_layers, n_layers, pl.hit_key,
                                                  pl.seg_off, pl.seg_fill, (BinnedHit*)pl.seg_rec,
                                                  pl.seg_bin);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // the largest layer's bin count, from the layout's per-layer bases
    int nb_max = 1;
    for (int l = 0; l < n_layers; ++l) {
        const int nb = (l + 1 < n_layers ? pl.bl.base[l + 1] : pl.bl.per_event) - pl.bl.base[l];
        if (nb > nb_max) nb_max = nb;
    }
    const size_t lds = sizeof(int) * ((size_t)nb_max + kBinSrcCap);
    bin_segment_kernel<<<(unsigned)n_seg, kBinThreads, lds, s>>>(
        pl.seg_off, (const BinnedHit*)pl.seg_rec, pl.seg_bin, d_layers, n_layers, (int)n_seg, nb_max,
        pl.bl, pl.off, (BinnedHit*)pl.binned);
    return hipGetLastError();
}

hipError_t launch_cost_order(const FindPlan& pl, const kf_tracks* seeds, int n_tiles,
                             int seeds_per_tile, hipStream_t s)
{
    if (seeds->n == 0) return launch_fill(pl.queue_loopers, kQueues, 0, s);
    const int64_t chunk = (int64_t)((n_tiles + kQueues - 1) / kQueues) * seeds_per_tile;
    const int nbq = (int)((chunk + kCostBlock - 1) / kCostBlock);
    cost_count_kernel<<<kQueues * nbq, kCostBlock, 0, s>>>(seeds->n, seeds->ld, (const float*)seeds->par,
                                                          pl.order, chunk, nbq, pl.cost_cnt);
    cost_place_kernel<<<kQueues * nbq, kCostBlock, 0, s>>>(seeds->n, seeds->ld, (const float*)seeds->par,
                                                          pl.order, chunk, nbq, pl.cost_cnt, pl.tile_order,
                                                          pl.queue_loopers);
    return hipGetLastError();
}

hipError_t launch_seed_order(const FindPlan& pl, const kf_tracks* seeds, const int32_t* seed_event,
                             const int32_t* event_off, int n_events, int largest_first,
                             hipStream_t s)
{
    if (seeds->n == 0) return hipSuccess;
    hipError_t e;
    const int64_t total = (int64_t)n_events * kSeedCells;
    if ((e = launch_fill(pl.scnt, total + 1, 0, s)) != hipSuccess) return e;
    // the ranking compares every pair of events: beyond kRankMaxEvents the
    // events keep their input order
    if (n_events > kRankMaxEvents) largest_first = 0;
    if (largest_first) {
        event_rank_kernel<<<blocks_for(n_events, 256), 256, 0, s>>>(event_off, n_events, pl.erank);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    seed_cell_kernel<<<blocks_for(seeds->n, 256), 256, 0, s>>>(
        seeds->n, seeds->ld, (const float*)seeds->par, seed_event, n_events,
        largest_first ? pl.erank : nullptr, pl.scnt, pl.cell);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_scan(pl.scnt, pl.soff, total + 1, pl.bsum, s)) != hipSuccess) return e;
    seed_scatter_kernel<<<blocks_for(seeds->n, 256), 256, 0, s>>>(seeds->n, pl.cell, pl.soff,
                                                                  pl.scnt, pl.order);
    cell_sort_kernel<<<blocks_for(total, 256), 256, 0, s>>>(total, pl.soff, pl.order);
    return hipGetLastError();
}

// ---------------------------------------------------------------- seed cleaning
// Duplicate seeds (same event; a shared hit, or eta, phi and q/pT all within
// the thresholds) and the order-free rule: a seed is removed iff a better
// duplicate exists.  Three passes: clear the claim slot of every hit a
// taking-part seed holds; in cell order, every seed writes a compact record
// (key, eta, phi, q/pT) at its position and claims its hits with an atomic
// minimum of its key; then, again in cell order, each seed checks its hits'
// claims (a lower key there is a better seed sharing that hit) and the
// records of its own and the eight neighbouring (eta, phi) cells, which are
// contiguous ranges (the thresholds are below a cell's width, so every
// parameter duplicate is there).

// (chi2 as float, then index), ascending = better; ~0 = takes no part
__device__ inline unsigned long long clean_key(float chi2, int64_t i)
{
    uint32_t u = __float_as_uint(chi2);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((unsigned long long)u << 32) | (unsigned long long)(uint32_t)i;
}

__device__ inline bool clean_part(uint32_t st, int32_t e, int n_events)
{
    return (st & kFreezeMask & ~(uint32_t)KF_ST_DUPLICATE) == 0 && e >= 0 && e < n_events;
}

__global__ __launch_bounds__(256) void clean_reset_kernel(int64_t n, int64_t ld,
                                                          const uint32_t* __restrict__ status,
                                                          const int32_t* __restrict__ seed_event,
                                                          int n_events,
                                                          const int32_t* __restrict__ seed_hits,
                                                          int64_t n_hits,
                                                          unsigned long long* __restrict__ best)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !clean_part(status[i], seed_event[i], n_events)) return;
    for (int k = 0; k < 3; ++k) {
        const int32_t h = seed_hits[k * ld + i];
        if (h >= 0 && h < n_hits) best[h] = ~0ull;
    }
}

__global__ __launch_bounds__(256) void clean_claim_kernel(
    int64_t n, int64_t ld, const float* __restrict__ par, const float* __restrict__ chi2,
    const uint32_t* __restrict__ status, const int32_t* __restrict__ seed_event, int n_events,
    const int32_t* __restrict__ seed_hits, int64_t n_hits, const int32_t* __restrict__ order,
    unsigned long long* __restrict__ best, CleanRec* __restrict__ rec)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t i = order[t];
    CleanRec r;
    if (!clean_part(status[i], seed_event[i], n_events)) {
        r.key = ~0ull;
        r.eta = 0.0;
        r.phi = 0.0f;
        r.c = 0.0f;
        rec[t] = r;
        return;
    }
    r.key = clean_key(chi2[i], i);
    r.eta = -log(tan(0.5 * (double)par[5 * ld + i]));
    r.phi = par[4 * ld + i];
    r.c = par[3 * ld + i];
    rec[t] = r;
    for (int k = 0; k < 3; ++k) {
        const int32_t h = seed_hits[k * ld + i];
        if (h >= 0 && h < n_hits) atomicMin(&best[h], r.key);
    }
}

__global__ __launch_bounds__(256) void clean_mark_kernel(
    int64_t n, int64_t ld, uint32_t* __restrict__ status, const int32_t* __restrict__ seed_hits,
    int64_t n_hits, const unsigned long long* __restrict__ best, const CleanRec* __restrict__ rec,
    const int32_t* __restrict__ cell, const int32_t* __restrict__ soff,
    const int32_t* __restrict__ order, double deta, double dphi, double dc)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const CleanRec me = rec[t];
    if (me.key == ~0ull) return;
    const int32_t j = order[t];
    bool dup = false;
    for (int k = 0; k < 3; ++k) {
        const int32_t h = seed_hits[k * ld + j];
        if (h >= 0 && h < n_hits && best[h] < me.key) dup = true;
    }
    if (!dup) {
        const double ej = me.eta, pj = me.phi, cj = me.c;
        const int c = cell[j];
        const int base = c - c % kSeedCells;
        const int fe = (c % kSeedCells) / 64, fp = c % 64;
        for (int de = -1; de <= 1 && !dup; ++de) {
            const int e2 = fe + de;
            if (e2 < 0 || e2 > 63) continue;
            for (int dp = -1; dp <= 1 && !dup; ++dp) {
                const int cc = base + e2 * 64 + ((fp + dp + 64) & 63);
                const int q1 = soff[cc + 1];
                for (int q = soff[cc]; q < q1; ++q) {
                    const CleanRec o = rec[q];
                    if (o.key >= me.key) continue;     // not better, itself, or no part
                    double d = (double)o.phi - pj;
                    if (d > kPi) d -= 2.0 * kPi;
                    if (d < -kPi) d += 2.0 * kPi;
                    if (fabs(o.eta - ej) < deta && fabs(d) < dphi && fabs((double)o.c - cj) < dc) {
                        dup = true;
                        break;
                    }
                }
            }
        }
    }
    const uint32_t st = status[j];
    status[j] = dup ? (st | (uint32_t)KF_ST_DUPLICATE) : (st & ~(uint32_t)KF_ST_DUPLICATE);
}

hipError_t launch_clean(const FindPlan& pl, const kf_tracks* seeds, const int32_t* seed_event,
                        int n_events, const int32_t* seed_hits, int64_t n_hits,
                        const kf_params& prm, hipStream_t s)
{
    if (seeds->n == 0) return hipSuccess;
    const unsigned nb = blocks_for(seeds->n, 256);
    clean_reset_kernel<<<nb, 256, 0, s>>>(seeds->n, seeds->ld, seeds->status, seed_event, n_events,
                                          seed_hits, n_hits, pl.clean_best);
    clean_claim_kernel<<<nb, 256, 0, s>>>(seeds->n, seeds->ld, (const float*)seeds->par,
                                          (const float*)seeds->chi2, seeds->status, seed_event,
                                          n_events, seed_hits, n_hits, pl.order, pl.clean_best,
                                          pl.clean_rec);
    clean_mark_kernel<<<nb, 256, 0, s>>>(seeds->n, seeds->ld, seeds->status, seed_hits, n_hits,
                                         pl.clean_best, pl.clean_rec, pl.cell, pl.soff, pl.order,
                                         prm.clean_deta, prm.clean_dphi, prm.clean_dc);
    return hipGetLastError();
}

// ---------------------------------------------------------------- duplicate removal
// Found tracks sharing at least frac of the shorter one's hits; the better by
// (more hits, lower float chi2, lower index) removes the other, each track
// decided independently.  A hit -> tracks index (count, prefix, scatter)
// limits the comparisons to tracks that meet in a hit; a pair's shared hits
// are counted layer by layer (a hit sits only in its own layer's column).

__device__ inline bool dedup_part(uint32_t st)
{
    return (st & kFreezeMask & ~(uint32_t)KF_ST_DUPTRACK) == 0;
}

__global__ __launch_bounds__(256) void dedup_count_kernel(int64_t n, int nl,
                                                          const int32_t* __restrict__ rows,
                                                          const uint32_t* __restrict__ status,
                                                          int64_t n_hits, int32_t* __restrict__ cnt,
                                                          int32_t* __restrict__ nh)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (!dedup_part(status[j])) {
        nh[j] = -1;
        return;
    }
    int c = 0;
    for (int l = 0; l < nl; ++l) {
        const int32_t h = rows[j * nl + l];
        if (h >= 0 && h < n_hits) {
            atomicAdd(&cnt[h], 1);
            ++c;
        }
    }
    nh[j] = c;
}

__global__ __launch_bounds__(256) void dedup_fill_kernel(int64_t n, int nl,
                                                         const int32_t* __restrict__ rows,
                                                         const int32_t* __restrict__ nh,
                                                         int64_t n_hits,
                                                         const int32_t* __restrict__ off,
                                                         int32_t* __restrict__ cnt,
                                                         int32_t* __restrict__ users)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n || nh[j] < 0) return;
    for (int l = 0; l < nl; ++l) {
        const int32_t h = rows[j * nl + l];
        if (h >= 0 && h < n_hits) users[off[h] + atomicSub(&cnt[h], 1) - 1] = (int32_t)j;
    }
}

// A track's shared-hit count with each partner is accumulated while walking
// its hits' user lists (a partner appears once per hit it shares); up to
// kDedupPartners better partners are tracked in registers, and a track with
// more falls back to counting each pair's shared hits layer by layer.
constexpr int kDedupPartners = 8;

__global__ __launch_bounds__(256) void dedup_mark_kernel(int64_t n, int nl,
                                                         const int32_t* __restrict__ rows,
                                                         const float* __restrict__ chi2,
                                                         uint32_t* __restrict__ status,
                                                         const int32_t* __restrict__ event,
                                                         const int32_t* __restrict__ nh,
                                                         int64_t n_hits,
                                                         const int32_t* __restrict__ off,
                                                         const int32_t* __restrict__ users,
                                                         double frac)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int nj = nh[j];
    if (nj < 0) return;
    const float fj = chi2[j];
    const int32_t ej = event[j];
    auto better = [&](int32_t i) {
        const int ni = nh[i];
        const float fi = chi2[i];
        return event[i] == ej && (ni > nj || (ni == nj && (fi < fj || (fi == fj && i < j))));
    };
    auto is_dup = [&](int32_t i, int shared) {
        const int ni = nh[i];
        const int mn = ni < nj ? ni : nj;
        return mn > 0 && (double)shared >= frac * (double)mn;
    };
    int32_t pid[kDedupPartners];
    int pcnt[kDedupPartners];
    int np = 0;
    bool overflow = false;
    for (int l = 0; l < nl; ++l) {
        const int32_t h = rows[j * nl + l];
        if (h < 0 || h >= n_hits) continue;
        for (int u = off[h]; u < off[h + 1]; ++u) {
            const int32_t i = users[u];
            if (i == j || !better(i)) continue;
            int q = 0;
#pragma unroll
            for (int r = 0; r < kDedupPartners; ++r)
                if (r < np && pid[r] == i) q = r + 1;
            if (q > 0) {
#pragma unroll
                for (int r = 0; r < kDedupPartners; ++r)
                    if (r == q - 1) ++pcnt[r];
            } else if (np < kDedupPartners) {
#pragma unroll
                for (int r = 0; r < kDedupPartners; ++r)
                    if (r == np) {
                        pid[r] = i;
                        pcnt[r] = 1;
                    }
                ++np;
            } else {
                overflow = true;
            }
        }
    }
    bool dup = false;
#pragma unroll
    for (int r = 0; r < kDedupPartners; ++r)
        if (r < np && is_dup(pid[r], pcnt[r])) dup = true;
    if (!dup && overflow) {
        // more better partners than tracked: count every pair directly
        for (int l = 0; l < nl && !dup; ++l) {
            const int32_t h = rows[j * nl + l];
            if (h < 0 || h >= n_hits) continue;
            for (int u = off[h]; u < off[h + 1] && !dup; ++u) {
                const int32_t i = users[u];
                if (i == j || !better(i)) continue;
                int shared = 0;
                for (int m = 0; m < nl; ++m) {
                    const int32_t hj = rows[j * nl + m];
                    shared += (hj >= 0 && hj < n_hits && rows[(int64_t)i * nl + m] == hj) ? 1 : 0;
                }
                dup = is_dup(i, shared);
            }
        }
    }
    const uint32_t st = status[j];
    status[j] = dup ? (st | (uint32_t)KF_ST_DUPTRACK) : (st & ~(uint32_t)KF_ST_DUPTRACK);
}

hipError_t launch_dedup(const FindPlan& pl, int64_t n, int nl, const int32_t* rows,
                        const float* chi2, uint32_t* status, const int32_t* event, int64_t n_hits,
                        double frac, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipError_t e;
    if ((e = launch_fill(pl.dup_cnt, n_hits + 1, 0, s)) != hipSuccess) return e;
    const unsigned nb = blocks_for(n, 256);
    dedup_count_kernel<<<nb, 256, 0, s>>>(n, nl, rows, status, n_hits, pl.dup_cnt, pl.dup_nh);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_scan(pl.dup_cnt, pl.dup_off, n_hits + 1, pl.bsum, s)) != hipSuccess) return e;
    dedup_fill_kernel<<<nb, 256, 0, s>>>(n, nl, rows, pl.dup_nh, n_hits, pl.dup_off, pl.dup_cnt,
                                         pl.dup_users);
    dedup_mark_kernel<<<nb, 256, 0, s>>>(n, nl, rows, chi2, status, event, pl.dup_nh, n_hits,
                                         pl.dup_off, pl.dup_users, frac);
    return hipGetLastError();
}

size_t plan_find(FindPlan* pl, void* base, int64_t n_hits, int n_events, int64_t n_seeds,
                 int n_layers, int grid, int seeds_per_tile)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? (void*)((char*)base + off) : nullptr;
        off += (bytes + 255) & ~size_t(255);
        return p;
    };
    const int64_t nb = (int64_t)n_events * pl->bl.per_event + 1;
    const int64_t nc = (int64_t)n_events * kSeedCells + 1;
    const int64_t ns = n_seeds > 0 ? n_seeds : 1;
    const int64_t nh = n_hits > 0 ? n_hits : 1;
    const int64_t nseg = (int64_t)n_events * n_layers + 1;
    int64_t nsmax = nseg > nc ? nseg : nc;
    if (nh + 1 > nsmax) nsmax = nh + 1;
    const int64_t nsum = (nsmax + kScanChunk - 1) / kScanChunk;
    pl->seg_cnt = (int32_t*)take(sizeof(int32_t) * 2 * nseg);
    pl->seg_fill = pl->seg_cnt + nseg;
    pl->seg_off = (int32_t*)take(sizeof(int32_t) * nseg);
    pl->off = (int32_t*)take(sizeof(int32_t) * nb);
    pl->hit_key = (int32_t*)take(sizeof(int32_t) * nh);
    pl->seg_rec = take(sizeof(BinnedHit) * nh);
    pl->seg_bin = (int32_t*)take(sizeof(int32_t) * nh);
    pl->binned = take(sizeof(BinnedHit) * nh);
    pl->scnt = (int32_t*)take(sizeof(int32_t) * nc);
    pl->soff = (int32_t*)take(sizeof(int32_t) * nc);
    pl->erank = (int32_t*)take(sizeof(int32_t) * n_events);
    pl->cell = (int32_t*)take(sizeof(int32_t) * ns);
    pl->order = (int32_t*)take(sizeof(int32_t) * ns);
    pl->tile_order = (int32_t*)take(sizeof(int32_t) * ns);
    {
        // class counts per block of the cost order, blocks as launch_cost_order makes them
        const int64_t S = seeds_per_tile > 0 ? seeds_per_tile : 1;
        const int64_t n_tiles = (ns + S - 1) / S;
        const int64_t chunk = (n_tiles + kQueues - 1) / kQueues * S;
        const int64_t nbq = (chunk + kCostBlock - 1) / kCostBlock;
        pl->cost_cnt = (int32_t*)take(sizeof(int32_t) * kCostClasses * kQueues * (size_t)nbq);
    }
    pl->queue_loopers = (int32_t*)take(sizeof(int32_t) * kQueues);
    pl->bsum = (int32_t*)take(sizeof(int32_t) * nsum);
    pl->bp = (int2*)take(sizeof(int2) * (size_t)grid * n_layers * seeds_per_tile * kMaxCands);
    pl->tile_counter = (int32_t*)take(sizeof(int32_t) * 64);
    pl->clean_best = (unsigned long long*)take(sizeof(unsigned long long) * nh);
    pl->clean_rec = (CleanRec*)take(sizeof(CleanRec) * ns);
    pl->dup_cnt = (int32_t*)take(sizeof(int32_t) * (nh + 1));
    pl->dup_off = (int32_t*)take(sizeof(int32_t) * (nh + 1));
    pl->dup_users = (int32_t*)take(sizeof(int32_t) * ns * (n_layers > 0 ? n_layers : 1));
    pl->dup_nh = (int32_t*)take(sizeof(int32_t) * ns);
    return off;
}

template <typename T, typename C, typename U, bool LEARN, bool MAT>
static void find_launch2(const FindArgs& a, int W, int grid, size_t lds, hipStream_t s)
{
    if (a.prm.field_z0 > 0.0) {
        if constexpr (!LEARN)
            if (a.steer) {
                find_kernel<T, C, U, false, MAT, true, true><<<grid, W, lds, s>>>(a);
                return;
            }
        find_kernel<T, C, U, LEARN, MAT, false, true><<<grid, W, lds, s>>>(a);
        return;
    }
    if constexpr (!LEARN)
        if (a.steer) {
            find_kernel<T, C, U, false, MAT, true, false><<<grid, W, lds, s>>>(a);
            return;
        }
    find_kernel<T, C, U, LEARN, MAT, false, false><<<grid, W, lds, s>>>(a);
}

template <typename T, typename C, typename U, bool LEARN>
static void find_launch(const FindArgs& a, int W, int grid, size_t lds, hipStream_t s)
{
    if (a.mat.x0)
        find_launch2<T, C, U, LEARN, true>(a, W, grid, lds, s);
    else
        find_launch2<T, C, U, LEARN, false>(a, W, grid, lds, s);
}

hipError_t launch_find_kernel(const FindArgs& a, int W, int grid, int prec, bool learn, hipStream_t s)
{
    const size_t lds = find_shared_size(W, a.seeds_per_tile, a.n_layers, prec);
    if (prec == KF_PREC_FP32)
        learn ? find_launch<float, float, float, true>(a, W, grid, lds, s)
              : find_launch<float, float, float, false>(a, W, grid, lds, s);
    else
        learn ? find_launch<float, double, double, true>(a, W, grid, lds, s)
              : find_launch<float, double, double, false>(a, W, grid, lds, s);
    return hipGetLastError();
}

}  // namespace kfmi
