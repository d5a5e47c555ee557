// Batched form of the spline path: many curves in CSR layout.
//
// Work of one run:
//   * build items: either one small curve per wavefront of the workgroup
//     (n <= 64*8), or one larger curve built by the whole workgroup
//     (n <= SOLVE_MAX_N_BATCH);
//   * evaluate slices: (curve, query range) pairs; a curve's queries are cut
//     into slices of at most queries_per_tile, fewer when its knots are
//     sparse relative to its queries (so that a slice's knots fit the staged
//     window), and never below one workgroup's worth.
// The fused kernel is persistent: each workgroup first claims build items
// with an atomic counter until none are left, then walks the tile list with a
// grid stride.  A tile waits (bounded spin) for its curve's ready flag.  This
// cannot deadlock at any grid size: a workgroup reaches the tiles only after
// every build item has been claimed, and a claimed item belongs to a
// workgroup that is running and waits on nothing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "spline_solve.h"

namespace spl {

constexpr int kItemLanes = 8;           // curves per packed build item (one per wavefront)
constexpr int kWaveBuildMaxN = 64 * 8;   // largest curve one wavefront builds
constexpr int kBatchWindow = 256;         // knots an evaluate slice stages
constexpr int32_t kItemPacked = 0;
constexpr int32_t kItemWhole = 1;

struct BuildItem {
    int32_t kind;               // kItemPacked: inst[w] is wavefront w's curve (-1 = none)
    int32_t inst[kItemLanes];   // kItemWhole: inst[0] is built by the whole workgroup
};

struct TileItem {  // uniform queries k0 .. k1-1 of curve inst
    int32_t inst;
    int32_t pad;
    int64_t k0;
    int64_t k1;
};

struct BatchDevArgs {
    const double* x;
    const double* y;
    const double* sd;
    const double* ed;
    const int64_t* koff;
    const int64_t* qoff;
    double* yq;
    double* ypp;
    int32_t* status;
    const BuildItem* items;
    const TileItem* tiles;
    int32_t* counters;  // [0] build item counter, [1] spin-timeout flag
    int32_t* ready;     // one flag per curve
    int32_t n_items;
    int32_t n_tiles;
    int32_t precision;
};

// Host side of a batch: the work tables and the device buffers that hold them.
class Batch {
public:
    explicit Batch(int device) : device_(device) {}
    ~Batch();
    Batch(const Batch&) = delete;
    Batch& operator=(const Batch&) = delete;

    // Plan from host offsets; returns a SOLVE_* code.  uniform (nullable):
    // per curve, 0 = no uniform evaluate tiles (its queries are evaluated by
    // another kernel; m may then be 0).
    int plan(int64_t count, const int64_t* koff, const int64_t* qoff, const spline_tuning& t, uint32_t precision,
             const uint8_t* uniform = nullptr);
    // Copy the tables to the device (async on s); the host tables must stay
    // alive until the copy completes (they are members, so until re-planning).
    int upload(hipStream_t s);
    // Same, through a caller-owned pinned staging buffer of table_bytes().
    int upload_staged(hipStream_t s, void* pinned);
    size_t table_bytes() const { return items_.size() * sizeof(BuildItem) + tiles_.size() * sizeof(TileItem); }
    // Launch one run on device-resident data.
    int launch(const double* x, const double* y, const double* sd, const double* ed, const int64_t* koff,
               const int64_t* qoff, double* yq, double* ypp, int32_t* status, hipStream_t s);

    int64_t count() const { return count_; }
    const spline_tuning& tuning() const { return tuning_; }
    void set_tuning(const spline_tuning& t) { tuning_ = t; }
    int retile(const spline_tuning& t);  // re-plan tiles for a new tile size
    int32_t spin_timeout_flag_host();    // synchronous read, for tests

    int device() const { return device_; }
    uint32_t precision() const { return precision_; }
    int64_t total_n() const { return total_n_; }
    int64_t total_m() const { return total_m_; }
    int32_t n_tiles() const { return (int32_t)tiles_.size(); }
    int32_t n_items() const { return (int32_t)items_.size(); }

private:
    int ensure(void** p, size_t* cap, size_t bytes);
    void make_tables();

    int device_;
    int64_t count_ = 0;
    int64_t total_n_ = 0, total_m_ = 0;
    uint32_t precision_ = 0;
    spline_tuning tuning_{};
    std::vector<int64_t> n_, m_;
    std::vector<uint8_t> uniform_;
    std::vector<BuildItem> items_;
    std::vector<TileItem> tiles_;
    void* d_items_ = nullptr;
    size_t cap_items_ = 0;
    void* d_tiles_ = nullptr;
    size_t cap_tiles_ = 0;
    void* d_counters_ = nullptr;  // counters (4 ints) then ready flags
    size_t cap_counters_ = 0;
    int num_cu_ = 0;
};

spline_tuning default_tuning();
bool valid_tuning(const spline_tuning& t);

}  // namespace spl
