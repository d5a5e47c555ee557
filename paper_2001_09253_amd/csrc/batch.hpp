// Batched form of the spline path: many curves in CSR layout.
//
// Phase 1 (only if the batch holds curves of at most kLaneBuildMaxN knots):
// 16 lanes per such curve (four curves per wavefront) solve it for y'': each
// lane runs the paper's sweeps over a chunk of rows and the chunks are joined
// by short scans.  Phase 2: a list of wave items, each run by
// one wavefront from start to end with no waiting on any other wavefront.  A
// wave item is (curve, knot block, query share): the wavefront stages the
// block's knots, values and y'' in its own LDS -- solving the span itself for
// curves past kLaneBuildMaxN knots: the whole curve when it fits one
// wavefront's rows, else the block of intervals plus a halo of rows on either
// side -- and then evaluates its share of the uniform queries that fall in the
// block.  Curves with many queries are cut into several shares so that no
// wavefront holds far more work than the average.  Items are ordered by
// decreasing work.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "spline_solve.h"

namespace spl {

constexpr uint8_t kCurveSkip = 2;    // Batch::plan: a curve the batch's kernels leave alone
constexpr int kLaneBuildMaxN = 256;  // curves up to this many knots are built in phase 1
constexpr int kMixedWaveMaxN = 512;  // mixed precision: curves up to this many knots take the lane-parallel build
constexpr int kBatchHalo = 128;      // halo rows on either side of a knot block
constexpr int kWaveMaxCH = 8;        // rows per lane of the largest wave span
constexpr int kWaveSpanMax = 64 * kWaveMaxCH;
constexpr int kWaveBlock = kWaveSpanMax - 1 - 2 * kBatchHalo;  // intervals per knot block

struct alignas(16) WaveItem {
    int64_t ko;     // first knot of the curve
    int64_t qo;     // first output of the curve
    int64_t m;      // its query count
    int32_t inst;   // curve
    int32_t n;      // its knot count
    int16_t j0;     // intervals [j0, j1) of the curve
    int16_t j1;
    int32_t s;      // share s of S of the block's queries (S = 0: y'' only)
    int32_t S;
    int32_t pad;
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
    const WaveItem* witems;
    int64_t n_witems;
    const int32_t* lane_curves;  // curves built in phase 1, longest first
    int64_t n_lane;
    int64_t prebuilt_max_n;      // curves up to this length were built in phase 1 (0: none)
    int32_t* bad;                // per curve, from phase 1: 1 if its knots are not increasing
    int32_t* idx;                // nullable: the interval of every query (CSR like yq, per curve)
};

// Host side of a batch: the work tables and the device buffers that hold them.
class Batch {
public:
    explicit Batch(int device) : device_(device) {}
    ~Batch();
    Batch(const Batch&) = delete;
    Batch& operator=(const Batch&) = delete;

    // Plan from host offsets; returns a SOLVE_* code.  uniform (nullable):
    // per curve, 0 = no uniform queries (y'' only: its queries are evaluated
    // by another kernel; m may then be 0), kCurveSkip = the batch's kernels
    // leave the curve alone (another launch solves it; any n >= 3).
    // host_only: build the work tables on the host only (no device buffer
    // is allocated; launch them with launch_with_tables and a `bad` buffer).
    int plan(int64_t count, const int64_t* koff, const int64_t* qoff, const spline_tuning& t, uint32_t precision,
             const uint8_t* uniform = nullptr, bool host_only = false);
    // Copy the tables to the device (async on s); the host tables must stay
    // alive until the copy completes (they are members, so until re-planning).
    int upload(hipStream_t s);
    // Bytes of the tables, and a copy of them into host memory at dst (in
    // the layout launch_with_tables expects).
    size_t table_bytes() const;
    void write_tables(void* dst) const;
    // Launch one run on device-resident data with the tables at the device
    // address tables (as written by write_tables), or with the plan's own
    // uploaded tables (launch).
    // idx (nullable): the interval of every query, written by the same
    // kernels compiled with the index store.
    int launch(const double* x, const double* y, const double* sd, const double* ed, const int64_t* koff,
               const int64_t* qoff, double* yq, double* ypp, int32_t* status, hipStream_t s, int32_t* idx = nullptr);
    // bad (nullable): per-curve flags of the phase-1 build (count int32),
    // instead of the plan's own buffer.
    int launch_with_tables(const void* tables, const double* x, const double* y, const double* sd,
                           const double* ed, const int64_t* koff, const int64_t* qoff, double* yq, double* ypp,
                           int32_t* status, hipStream_t s, int32_t* idx = nullptr, int32_t* bad = nullptr);
    // Whether the launch needs the per-curve `bad` flags (a phase-1 build).
    bool needs_bad() const { return !lane_.empty(); }

    int64_t count() const { return count_; }
    const spline_tuning& tuning() const { return tuning_; }
    int retile(const spline_tuning& t);  // re-plan for new tuning

    int device() const { return device_; }
    uint32_t precision() const { return precision_; }
    int64_t total_n() const { return total_n_; }
    int64_t total_m() const { return total_m_; }
    int64_t n_witems() const { return (int64_t)witems_.size(); }
    int64_t n_lane() const { return (int64_t)lane_.size(); }
    int wave_rows() const { return wave_ch_ * 64; }

private:
    int ensure(void** p, size_t* cap, size_t bytes);
    void make_tables();

    int device_;
    int64_t count_ = 0;
    int64_t total_n_ = 0, total_m_ = 0;
    int64_t max_n_ = 0;
    int wave_ch_ = 1;
    uint32_t precision_ = 0;
    spline_tuning tuning_{};
    std::vector<int64_t> n_, m_, koff_, qoff_;
    std::vector<uint8_t> uniform_;
    std::vector<WaveItem> witems_;
    std::vector<int32_t> lane_;
    int64_t lane_max_n_ = 0;
    int64_t lane_long_ = 0;  // leading lane_ entries past kMixedWaveMaxN knots (mixed precision)
    int64_t prebuilt_max_n_ = 0;
    void* d_bad_ = nullptr;
    size_t cap_bad_ = 0;
    size_t offset_lane() const;
    void* d_tables_ = nullptr;
    size_t cap_tables_ = 0;
    int num_cu_ = 0;
};

spline_tuning default_tuning();
bool valid_tuning(const spline_tuning& t);

}  // namespace spl
