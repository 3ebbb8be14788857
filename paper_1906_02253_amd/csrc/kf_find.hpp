// Internal interface of the finding kernels (kf_find.hip) for the C-ABI layer.
#pragma once

#include "kf_internal.hpp"

namespace kfmi {

constexpr int kMaxCands = 8;    // candidate slots per seed the kernel is built for
constexpr int kMaxLayerBins = 16384;   // nbin_phi * nbin_2 of one layer (LDS histogram)
constexpr int kFindCounters = 8;       // event counters of a finding call

// Seeds per workgroup of the finding kernel: max_cands lanes per seed, and a
// seed never straddles two waves (its candidates exchange state by shuffles).
__host__ __device__ inline int seeds_per_wave(int W, int MC) { return (W < 64 ? W : 64) / MC; }
__host__ __device__ inline int seeds_per_wg(int W, int MC)
{
    return W < 64 ? W / MC : (W / 64) * (64 / MC);
}

// One binned hit: position, sigmas, azimuth cos/sin and the caller's hit index.
struct alignas(16) BinnedHit {
    float x, y, z, su;
    float sv, cphi, sphi;
    int32_t idx;
};

// Bin layout of one event: layer l owns bins [base[l], base[l] + nbin_phi*nbin_2),
// phi-major; events are per_event bins apart.
struct BinLayout {
    int32_t base[kMaxLayers];
    int32_t per_event;
};

struct FindArgs {
    // binned hits of all events
    const BinnedHit* bh;
    const int32_t* bin_off;
    BinLayout bl;
    int64_t n_hits;
    const int32_t* hit_layer;
    // seeds (par/cov/chi2/ndf/status after the seed fit), SoA with leading dim sld
    int64_t n_seeds, sld;
    const float* spar;
    const float* scov;            // float storage (mixed and FP32 modes)
    const float* schi2;
    const int32_t* sndf;
    const uint32_t* sstatus;
    const int32_t* seed_event;
    int n_events;
    const int32_t* seed_hits;     // [3][sld]
    const int32_t* order;         // seeds in processing order
    // outputs
    int32_t* out_hits;            // [n_seeds][n_layers]
    int64_t old;
    float* opar;
    float* ocov;
    float* ochi2;
    int32_t* ondf;
    uint32_t* ostatus;
    // scratch
    int2* bp;                     // per workgroup: [n_layers][S][kMaxCands] back-pointers
    int32_t* tile_counter;
    const int32_t* queue_loopers; // [kQueues] costliest-class seeds at the head of each tile
                                  // queue's range (served in sparser tiles)
    unsigned long long* counters; // optional [kFindCounters]: propagations, updates, chi2 tests,
                                  // Newton evaluations, disk tests, learned guesses, fallbacks,
                                  // children kept from propagated parents
    // geometry and parameters
    const kf_layer* layers;
    int n_layers;
    kf_params prm;
    int material;
    int n_tiles;
    int seeds_per_tile;
    MatMap mat;                   // r-z material map (x0 == nullptr: none)
    const SteerDev* steer;        // tracking regions and plans (nullptr: dynamic navigation)
    MlpDev mlp;                   // learned guess (KF_INIT_MLP)
};

// Device scratch of one kf_find call, carved from the context workspace.
// A seed as the cleaning compares it, stored at its position in cell order:
// key = (chi2 as float, index), ~0 when the seed takes no part.
struct CleanRec {
    unsigned long long key;
    double eta;
    float phi, c;
};

struct FindPlan {
    BinLayout bl;
    int32_t* seg_cnt;   // [n_events * n_layers + 1] hits per (event, layer) segment
    int32_t* seg_fill;  // [n_events * n_layers + 1] hits placed per segment so far
    int32_t* seg_off;   // [n_events * n_layers + 1] exclusive prefix sum of seg_cnt
    int32_t* off;       // [n_events * per_event + 1] first binned hit of every bin
    int32_t* hit_key;   // [n_hits] segment of each hit (-1: not binned)
    void* seg_rec;      // [n_hits] hit records grouped by segment (32 bytes each)
    int32_t* seg_bin;   // [n_hits] bin of each grouped record within its layer
    void* binned;       // [n_hits] records of 32 bytes
    int32_t* scnt;      // [n_events * cells + 1] seeds per (event, eta, phi) cell
    int32_t* soff;      // [n_events * cells + 1] its exclusive prefix sum
    int32_t* erank;     // [n_events] processing position of each event
    int32_t* cell;      // [n_seeds] cell of each seed
    int32_t* order;     // [n_seeds] seeds in (event, eta, phi) cell order
    int32_t* tile_order;  // [n_seeds] the finding kernel's order: the cell order partitioned
                          // by cost class inside each tile queue's range
    int32_t* cost_cnt;  // [kQueues][blocks][classes] cost classes per block of the tile order
    int32_t* queue_loopers;  // [kQueues] seeds of the costliest class in each queue's range
    int32_t* bsum;      // chunk totals of the prefix sums
    int2* bp;
    int32_t* tile_counter;
    unsigned long long* clean_best;  // [n_hits] best seed claiming each hit (seed cleaning)
    CleanRec* clean_rec;      // [n_seeds] cleaning records in seed (cell) order
    int32_t* dup_cnt;         // [n_hits + 1] tracks per hit (duplicate removal)
    int32_t* dup_off;         // [n_hits + 1] its exclusive prefix sum
    int32_t* dup_users;       // [n_seeds * n_layers] tracks of each hit, grouped by hit
    int32_t* dup_nh;          // [n_seeds] hits per taking-part track, -1 = no part
};

// Lays out the scratch of a call from `base` (nullptr: only sizes it); returns bytes.
size_t plan_find(FindPlan* pl, void* base, int64_t n_hits, int n_events, int64_t n_seeds,
                 int n_layers, int grid, int seeds_per_tile);
size_t find_shared_size(int W, int S, int nl, int prec);
hipError_t find_max_blocks_per_cu(int W, int S, int nl, int prec, bool learn, bool mat, bool steer,
                                  bool field, int* out);
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* bsum, hipStream_t s);
hipError_t launch_fill(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_bin(const FindPlan& pl, const kf_hits* h, const int32_t* event_off, int n_events,
                      const kf_layer* d_layers, int n_layers, hipStream_t s);
// Seed cleaning over the cells the seed order just built (pl.cell, pl.soff,
// pl.order): marks or clears KF_ST_DUPLICATE in seeds->status.
hipError_t launch_clean(const FindPlan& pl, const kf_tracks* seeds, const int32_t* seed_event,
                        int n_events, const int32_t* seed_hits, int64_t n_hits,
                        const kf_params& prm, hipStream_t s);
// Duplicate removal of found tracks: marks or clears KF_ST_DUPTRACK in status.
hipError_t launch_dedup(const FindPlan& pl, int64_t n, int nl, const int32_t* rows,
                        const float* chi2, uint32_t* status, const int32_t* event, int64_t n_hits,
                        double frac, hipStream_t s);
// The finding kernel's tile order (pl.tile_order) from the cell order.
hipError_t launch_cost_order(const FindPlan& pl, const kf_tracks* seeds, int n_tiles,
                             int seeds_per_tile, hipStream_t s);
hipError_t launch_seed_order(const FindPlan& pl, const kf_tracks* seeds, const int32_t* seed_event,
                             const int32_t* event_off, int n_events, int largest_first,
                             hipStream_t s);
hipError_t launch_find_kernel(const FindArgs& a, int W, int grid, int prec, bool learn, hipStream_t s);

}  // namespace kfmi
