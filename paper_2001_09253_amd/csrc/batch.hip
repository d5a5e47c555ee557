// Batched spline path: the single-launch wave-item kernel, hipGraph capture
// and the autotuner (C ABI: spline_plan_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <numeric>
#include <sstream>
#include <string>

#include "batch.hpp"
#include "spline_kernels.hpp"
#include "spline_solve.h"

namespace spl {

struct alignas(16) IntervalConst {  // 1/(b - a) and (b - a)^2 of one interval
    double inv, ba2;
};

// One wavefront's LDS: the span's knots, values and second derivatives (knot j
// at [j - max(rs - 1, 0)], y'' of row j at so[j - rs]) and the constants of the
// owned intervals (interval t at ib[t - j0]).
template <int CH>
struct WaveSmem {
    static constexpr int kRows = kWave * CH;
    double sx[kRows + 2];
    double sy[kRows + 2];
    double so[kRows + 2];
    IntervalConst ib[kRows];
};

// Whether x[0..n) fails to increase strictly (or holds a NaN); every lane of
// the wavefront gets the answer.
__device__ __forceinline__ bool wave_unordered(const double* __restrict__ x, int n, int lane) {
    bool bad = false;
    for (int j = 1 + lane; j < n; j += kWave) bad |= !(x[j] > x[j - 1]);
    return __ballot(bad) != 0ull;
}

// One wave item.  All 64 lanes of the wavefront call this.
template <int CH>
__device__ void run_wave_item(const BatchDevArgs& a, const WaveItem it, WaveSmem<CH>& sm, int lane) {
    const int i = it.inst;
    const int64_t ko = a.koff[i];
    const int n = (int)(a.koff[i + 1] - ko);
    const int64_t qo = a.qoff[i];
    const int64_t m = a.qoff[i + 1] - qo;
    const double* __restrict__ x = a.x + ko;
    const double* __restrict__ y = a.y + ko;
    const int j0 = it.j0;
    const int j1 = it.j1;
    const bool whole = j0 == 0 && j1 == n - 1;
    const bool reporter = j0 == 0 && it.s == 0;  // writes the curve's status (and NaNs if it is bad)
    // a1-a4: y'' over the span, exact for a whole curve and exact to rounding
    // with the halo (the dropped coupling decays by 2/3 or better per row).
    const int rs = whole ? 0 : max(0, j0 - kBatchHalo);
    const int re = whole ? n : min(n, j1 + 1 + kBatchHalo);
    bool bad = build_span<kWave, CH, true, SoloGroup, true>(x, y, n, rs, re, a.sd[i], a.ed[i], nullptr, nullptr,
                                                             sm.sx, nullptr, nullptr, SoloGroup{}, lane, sm.sy,
                                                             sm.so);
    if (!whole) bad = bad || wave_unordered(x, n, lane);
    if (bad) {
        if (reporter) {
            const double nan = __builtin_nan("");
            if (a.ypp)
                for (int j = lane; j < n; j += kWave) a.ypp[ko + j] = nan;
            if (it.S > 0)
                for (int64_t k = lane; k < m; k += kWave) a.yq[qo + k] = nan;
            if (a.status && lane == 0) a.status[i] = kStatusOrder;
        }
        return;
    }
    if (reporter && a.status && lane == 0) a.status[i] = kStatusOk;
    const int lo = max(rs - 1, 0);
    if (it.s == 0 && a.ypp) {
        const int jend = j1 + (j1 == n - 1 ? 1 : 0);  // the last block also owns the last knot
        for (int j = j0 + lane; j < jend; j += kWave) a.ypp[ko + j] = sm.so[j - rs];
    }
    if (it.S == 0) return;
    for (int t = j0 + lane; t < j1; t += kWave) {
        const double ba = sm.sx[t + 1 - lo] - sm.sx[t - lo];
        sm.ib[t - j0] = IntervalConst{1.0 / ba, ba * ba};
    }
    wave_sync();

    // a5: the block's queries are those in (x_j0, x_j1] (from k = 0 for the
    // first block); this item takes share s of S of them.
    const double x0 = x[0];
    const double xl = x[n - 1];
    const double h = uniform_step(x0, xl, m);
    const double rh = (m > 1) ? 1.0 / h : 0.0;
    const int64_t ka = (j0 == 0) ? 0 : first_query_above_r(x0, xl, h, rh, m, sm.sx[j0 - lo]);
    const int64_t kb = (j1 == n - 1) ? m : first_query_above_r(x0, xl, h, rh, m, sm.sx[j1 - lo]);
    const int64_t len = kb - ka;
    const int64_t per = len / it.S;
    const int64_t rem = len % it.S;
    const int64_t k0 = ka + per * it.s + min((int64_t)it.s, rem);
    const int64_t k1 = k0 + per + ((int64_t)it.s < rem ? 1 : 0);
    if (k0 >= k1) return;
    double* __restrict__ out = a.yq + qo;

    if (len < 4 * (int64_t)(j1 - j0)) {
        // sparse: every query searches the block's knots
        for (int64_t k = k0 + lane; k < k1; k += kWave) {
            const double q = uniform_query(x0, xl, h, m, k);
            const int t = (int)lower_bound_idx(sm.sx, j0 + 1 - lo, j1 - 1 - j0, q) + lo - 1;
            const IntervalConst c = sm.ib[t - j0];
            out[k] = newint(q, sm.sx[t - lo], sm.sx[t + 1 - lo], sm.sy[t - lo], sm.sy[t + 1 - lo],
                            sm.so[t - rs], sm.so[t + 1 - rs], c.inv);
        }
        return;
    }
    // dense: 64 consecutive queries at a time; the wavefront carries the
    // interval t of its next query and the first query knext of interval
    // t + 1, and each lane moves past the boundaries its own query crossed.
    int t = j0;
    if (k0 > ka) {
        // interval of query k0: j0 plus the interior knots of the block below it
        const double q0 = uniform_query(x0, xl, h, m, k0);
        int cnt = 0;
        for (int j = j0 + 1 + lane; j - lane < j1; j += kWave)
            cnt += __popcll(__ballot(j < j1 && sm.sx[j - lo] < q0));
        t = j0 + cnt;
    }
    int64_t knext = (t + 1 < j1) ? first_query_above_r(x0, xl, h, rh, m, sm.sx[t + 1 - lo]) : k1;
    const double dl = (double)lane;
    for (int64_t kc = k0; kc < k1; kc += kWave) {
        const int64_t k = kc + lane;
        const int64_t klast = min(kc + kWave - 1, k1 - 1);
        int tl = t;
        while (knext <= klast) {
            ++t;
            tl = (k >= knext) ? t : tl;
            knext = (t + 1 < j1) ? first_query_above_r(x0, xl, h, rh, m, sm.sx[t + 1 - lo]) : k1;
        }
        if (k < k1) {
            double q;
            {
#pragma clang fp contract(off)
                // (double)kc + lane is (double)k exactly: the position equals
                // uniform_query(.., k) bit for bit
                const double step = ((double)kc + dl) * h;
                q = x0 + step;
            }
            q = (k >= m - 1) ? xl : q;
            q = (k <= 0) ? x0 : q;
            const IntervalConst c = sm.ib[tl - j0];
            const double av = sm.sx[tl - lo];
            const double bv = sm.sx[tl + 1 - lo];
            // a6: newint with the interval's 1/(b - a) and (b - a)^2
            const double xa = q - av;
            const double bx = bv - q;
            const double lower = xa * sm.sy[tl + 1 - lo] + bx * sm.sy[tl - lo];
            const double C = (xa * xa - c.ba2) * xa * sm.so[tl + 1 - rs];
            const double D = (bx * bx - c.ba2) * bx * sm.so[tl - rs];
            out[k] = (lower + (1.0 / 6.0) * (C + D)) * c.inv;
        }
    }
}

template <int CH, int WPG>
__global__ __launch_bounds__(WPG * kWave) void wave_items_kernel(BatchDevArgs a) {
    __shared__ WaveSmem<CH> smem[WPG];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int64_t stride = (int64_t)gridDim.x * WPG;
    for (int64_t w = (int64_t)blockIdx.x * WPG + wid; w < a.n_witems; w += stride)
        run_wave_item<CH>(a, a.witems[w], smem[wid], lane);
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

static int wave_ch_for(int64_t max_n) {
    if (max_n <= 64) return 1;
    if (max_n <= 128) return 2;
    if (max_n <= 192) return 3;
    if (max_n <= 256) return 4;
    return kWaveMaxCH;
}

template <int CH, int WPG>
static int launch_waves(const BatchDevArgs& a, int grid_per_cu, int num_cu, hipStream_t s) {
    const int64_t groups = (a.n_witems + WPG - 1) / WPG;
    int64_t grid = groups;
    if (grid_per_cu > 0) grid = std::min<int64_t>(groups, (int64_t)num_cu * grid_per_cu);
    if (grid < 1) return SOLVE_OK;
    wave_items_kernel<CH, WPG><<<(unsigned)grid, WPG * kWave, 0, s>>>(a);
    return SOLVE_OK;
}

template <int CH>
static int launch_waves_ch(const BatchDevArgs& a, const spline_tuning& t, int num_cu, hipStream_t s) {
    switch (t.block) {
        case 64: return launch_waves<CH, 1>(a, t.grid_per_cu, num_cu, s);
        case 128: return launch_waves<CH, 2>(a, t.grid_per_cu, num_cu, s);
        case 256: return launch_waves<CH, 4>(a, t.grid_per_cu, num_cu, s);
        default: return SOLVE_E_ARG;
    }
}

spline_tuning default_tuning() {
    spline_tuning t;
    t.block = 256;
    t.queries_per_tile = 4096;
    t.grid_per_cu = 0;
    t.fused = 1;
    return t;
}

bool valid_tuning(const spline_tuning& t) {
    return t.fused == 1 && (t.block == 64 || t.block == 128 || t.block == 256) && t.queries_per_tile >= 64 &&
           t.queries_per_tile <= (1 << 24) && t.grid_per_cu >= 0 && t.grid_per_cu <= 64;
}

Batch::~Batch() { (void)hipFree(d_tables_); }

int Batch::ensure(void** p, size_t* cap, size_t bytes) {
    if (bytes <= *cap && *p) return SOLVE_OK;
    size_t want = std::max<size_t>(bytes, 256);
    want = std::max(want, *cap + *cap / 2);
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc(p, want) != hipSuccess) {
        *p = nullptr;
        return SOLVE_E_DEVICE;
    }
    *cap = want;
    return SOLVE_OK;
}

void Batch::make_tables() {
    // wave items: whole curves when they fit one wavefront's rows, else knot
    // blocks with halos; shares of at most about queries_per_tile queries
    witems_.clear();
    const int rows = wave_ch_ * kWave;
    const int64_t cap = tuning_.queries_per_tile;
    std::vector<double> cost;
    for (int64_t i = 0; i < count_; ++i) {
        const int64_t n = n_[i];
        const int bk = (n <= rows) ? (int)(n - 1) : kWaveBlock;
        for (int64_t j0 = 0; j0 < n - 1; j0 += bk) {
            const int64_t j1 = std::min<int64_t>(j0 + bk, n - 1);
            const int64_t span = (n <= rows) ? n : std::min<int64_t>(n, j1 + 1 + kBatchHalo) -
                                                       std::max<int64_t>(0, j0 - kBatchHalo);
            int64_t S = 0;
            double est = 0.0;
            if (uniform_[i]) {
                est = (double)m_[i] * (double)(j1 - j0) / (double)(n - 1);
                S = std::max<int64_t>(1, (int64_t)std::ceil(est / (double)cap));
            }
            for (int64_t s = 0; s < std::max<int64_t>(S, 1); ++s) {
                witems_.push_back(WaveItem{(int32_t)i, (int16_t)j0, (int16_t)j1, (int32_t)s, (int32_t)S});
                // a row of the build costs about as much as 8 queries
                cost.push_back(8.0 * (double)span + (S ? est / (double)S : 0.0));
            }
        }
    }
    // decreasing work, so that the last wavefronts to start hold the least
    std::vector<size_t> order(witems_.size());
    std::iota(order.begin(), order.end(), (size_t)0);
    std::stable_sort(order.begin(), order.end(), [&](size_t p, size_t q) { return cost[p] > cost[q]; });
    std::vector<WaveItem> sorted(witems_.size());
    for (size_t k = 0; k < order.size(); ++k) sorted[k] = witems_[order[k]];
    witems_.swap(sorted);
}

int Batch::plan(int64_t count, const int64_t* koff, const int64_t* qoff, const spline_tuning& t,
                uint32_t precision, const uint8_t* uniform) {
    if (count < 1 || !koff || !qoff) return SOLVE_E_ARG;
    if (count > 0x7fffffffLL) return SOLVE_E_SIZE;
    if (!valid_tuning(t)) return SOLVE_E_ARG;
    if (precision != SOLVE_FP64) return SOLVE_E_ARG;
    if (koff[0] != 0 || qoff[0] != 0) return SOLVE_E_ARG;
    n_.assign(count, 0);
    m_.assign(count, 0);
    uniform_.assign(count, 1);
    max_n_ = 0;
    for (int64_t i = 0; i < count; ++i) {
        n_[i] = koff[i + 1] - koff[i];
        m_[i] = qoff[i + 1] - qoff[i];
        if (uniform) uniform_[i] = uniform[i] ? 1 : 0;
        if (n_[i] < 3 || n_[i] > SOLVE_MAX_N_BATCH || m_[i] < (uniform_[i] ? 1 : 0)) return SOLVE_E_SIZE;
        max_n_ = std::max(max_n_, n_[i]);
    }
    count_ = count;
    total_n_ = koff[count];
    total_m_ = qoff[count];
    precision_ = precision;
    if (!num_cu_) {
        if (hipDeviceGetAttribute(&num_cu_, hipDeviceAttributeMultiprocessorCount, device_) != hipSuccess)
            return SOLVE_E_DEVICE;
    }
    return retile(t);
}

int Batch::retile(const spline_tuning& t) {
    if (!valid_tuning(t)) return SOLVE_E_ARG;
    tuning_ = t;
    wave_ch_ = wave_ch_for(max_n_);
    make_tables();
    return ensure(&d_tables_, &cap_tables_, table_bytes());
}

size_t Batch::table_bytes() const { return witems_.size() * sizeof(WaveItem); }

void Batch::write_tables(void* dst) const {
    if (!witems_.empty()) std::memcpy(dst, witems_.data(), table_bytes());
}

int Batch::upload(hipStream_t s) {
    if (!witems_.empty() &&
        hipMemcpyAsync(d_tables_, witems_.data(), table_bytes(), hipMemcpyHostToDevice, s) != hipSuccess)
        return SOLVE_E_DEVICE;
    return SOLVE_OK;
}

int Batch::launch(const double* x, const double* y, const double* sd, const double* ed, const int64_t* koff,
                  const int64_t* qoff, double* yq, double* ypp, int32_t* status, hipStream_t s) {
    return launch_with_tables(d_tables_, x, y, sd, ed, koff, qoff, yq, ypp, status, s);
}

int Batch::launch_with_tables(const void* tables, const double* x, const double* y, const double* sd,
                              const double* ed, const int64_t* koff, const int64_t* qoff, double* yq, double* ypp,
                              int32_t* status, hipStream_t s) {
    if (!tables || !x || !y || !sd || !ed || !koff || !qoff || !yq || !ypp) return SOLVE_E_ARG;
    BatchDevArgs a;
    a.x = x;
    a.y = y;
    a.sd = sd;
    a.ed = ed;
    a.koff = koff;
    a.qoff = qoff;
    a.yq = yq;
    a.ypp = ypp;
    a.status = status;
    a.witems = (const WaveItem*)tables;
    a.n_witems = (int64_t)witems_.size();
    int rc = SOLVE_E_ARG;
    switch (wave_ch_) {
        case 1: rc = launch_waves_ch<1>(a, tuning_, num_cu_, s); break;
        case 2: rc = launch_waves_ch<2>(a, tuning_, num_cu_, s); break;
        case 3: rc = launch_waves_ch<3>(a, tuning_, num_cu_, s); break;
        case 4: rc = launch_waves_ch<4>(a, tuning_, num_cu_, s); break;
        case kWaveMaxCH: rc = launch_waves_ch<kWaveMaxCH>(a, tuning_, num_cu_, s); break;
        default: break;
    }
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

}  // namespace spl

using namespace spl;

struct spline_plan {
    Batch batch;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    explicit spline_plan(int dev) : batch(dev) {}
    ~spline_plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
    }
};

std::string arch_name(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string s = p.gcnArchName;
    const size_t c = s.find(':');
    return c == std::string::npos ? s : s.substr(0, c);
}

std::string size_class(const Batch& b) {
    const double mn = (double)b.total_n() / (double)b.count();
    const double mm = (double)b.total_m() / (double)b.count();
    char buf[128];
    snprintf(buf, sizeof buf, "c%d_n%d_m%d_p%u", (int)std::lround(std::log2((double)b.count())),
             (int)std::lround(std::log2(mn)), (int)std::lround(std::log2(mm)), b.precision());
    return buf;
}

// Minimal flat JSON object store: {"key": [block, q, grid_per_cu, fused, ms], ...}
std::map<std::string, std::vector<double>> read_cache(const char* path) {
    std::map<std::string, std::vector<double>> out;
    if (!path) return out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t pos = 0;
    while ((pos = t.find('"', pos)) != std::string::npos) {
        const size_t e = t.find('"', pos + 1);
        if (e == std::string::npos) break;
        const std::string key = t.substr(pos + 1, e - pos - 1);
        const size_t lb = t.find('[', e), rb = t.find(']', e);
        if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
        std::vector<double> v;
        std::stringstream vs(t.substr(lb + 1, rb - lb - 1));
        std::string tok;
        while (std::getline(vs, tok, ',')) v.push_back(std::atof(tok.c_str()));
        out[key] = v;
        pos = rb + 1;
    }
    return out;
}

void write_cache(const char* path, const std::map<std::string, std::vector<double>>& c) {
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << "{\n";
        size_t k = 0;
        for (const auto& kv : c) {
            f << "  \"" << kv.first << "\": [";
            for (size_t i = 0; i < kv.second.size(); ++i) f << (i ? ", " : "") << kv.second[i];
            f << "]" << (++k < c.size() ? "," : "") << "\n";
        }
        f << "}\n";
    }
    std::rename(tmp.c_str(), path);
}

}  // namespace

extern "C" int spline_plan_create(int device, int64_t count, const int64_t* koff, const int64_t* qoff,
                                  uint32_t precision, const spline_tuning* tuning, spline_plan** out) {
    if (!out || !koff || !qoff) return SOLVE_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SOLVE_E_DEVICE;
    DeviceGuard g(device);
    spline_plan* p = new spline_plan(device);
    const spline_tuning t = tuning ? *tuning : default_tuning();
    int rc = p->batch.plan(count, koff, qoff, t, precision);
    if (!rc) rc = p->batch.upload(nullptr);
    if (!rc && hipStreamSynchronize(nullptr) != hipSuccess) rc = SOLVE_E_DEVICE;
    if (rc) {
        delete p;
        return rc;
    }
    *out = p;
    return SOLVE_OK;
}

extern "C" int spline_plan_run(spline_plan* p, const double* x, const double* y, const double* sd,
                               const double* ed, const int64_t* koff, const int64_t* qoff, double* yq,
                               double* ypp, int32_t* status, void* stream) {
    if (!p) return SOLVE_E_ARG;
    DeviceGuard g(p->batch.device());
    return p->batch.launch(x, y, sd, ed, koff, qoff, yq, ypp, status, (hipStream_t)stream);
}

extern "C" int spline_plan_capture(spline_plan* p, const double* x, const double* y, const double* sd,
                                   const double* ed, const int64_t* koff, const int64_t* qoff, double* yq,
                                   double* ypp, int32_t* status, void* stream) {
    if (!p) return SOLVE_E_ARG;
    DeviceGuard g(p->batch.device());
    hipStream_t s = (hipStream_t)stream;
    hipStream_t cs = nullptr;
    if (!s) {
        // the legacy stream cannot be captured: capture on a private stream
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return SOLVE_E_DEVICE;
        s = cs;
    }
    if (p->exec) { (void)hipGraphExecDestroy(p->exec); p->exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    int rc = SOLVE_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = SOLVE_E_DEVICE;
    if (!rc) {
        const int lrc = p->batch.launch(x, y, sd, ed, koff, qoff, yq, ypp, status, s);
        hipGraph_t gr = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &gr);
        if (lrc) rc = lrc;
        else if (e != hipSuccess || !gr) rc = SOLVE_E_DEVICE;
        if (gr && rc) (void)hipGraphDestroy(gr);
        if (!rc) {
            p->graph = gr;
            if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
                p->exec = nullptr;
                rc = SOLVE_E_DEVICE;
            }
        }
    }
    if (cs) (void)hipStreamDestroy(cs);
    return rc;
}

extern "C" int spline_plan_replay(spline_plan* p, void* stream) {
    if (!p || !p->exec) return SOLVE_E_ARG;
    DeviceGuard g(p->batch.device());
    return hipGraphLaunch(p->exec, (hipStream_t)stream) == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

extern "C" int spline_plan_get_tuning(const spline_plan* p, spline_tuning* out) {
    if (!p || !out) return SOLVE_E_ARG;
    *out = p->batch.tuning();
    return SOLVE_OK;
}

extern "C" int spline_plan_autotune(spline_plan* p, const double* x, const double* y, const double* sd,
                                    const double* ed, const int64_t* koff, const int64_t* qoff, double* yq,
                                    double* ypp, int reps, const char* cache_path, spline_tuning* best,
                                    double* best_ms) {
    if (!p || !best || !best_ms) return SOLVE_E_ARG;
    if (reps < 1) reps = 1;
    DeviceGuard g(p->batch.device());
    Batch& b = p->batch;
    const std::string key = arch_name(b.device()) + ":" + size_class(b);
    auto cache = read_cache(cache_path);
    auto hit = cache.find(key);
    if (hit != cache.end() && hit->second.size() >= 5) {
        spline_tuning t;
        t.block = (int32_t)hit->second[0];
        t.queries_per_tile = (int32_t)hit->second[1];
        t.grid_per_cu = (int32_t)hit->second[2];
        t.fused = (int32_t)hit->second[3];
        if (valid_tuning(t)) {
            int rc = b.retile(t);
            if (!rc) rc = b.upload(nullptr);
            if (!rc && hipStreamSynchronize(nullptr) != hipSuccess) rc = SOLVE_E_DEVICE;
            if (rc) return rc;
            *best = t;
            *best_ms = hit->second[4];
            return SOLVE_OK;
        }
    }
    // wavefronts per workgroup x query share x (one item per wavefront, or
    // persistent wavefronts)
    std::vector<spline_tuning> cands;
    for (int block : {64, 128, 256})
        for (int cap : {1024, 2048, 4096, 8192})
            for (int gpc : {0, 16}) cands.push_back(spline_tuning{block, cap, gpc, 1});
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return SOLVE_E_DEVICE;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double bms = 1e300;
    spline_tuning bt = b.tuning();
    int rc = SOLVE_OK;
    for (const auto& t : cands) {
        rc = b.retile(t);
        if (!rc) rc = b.upload(s);
        for (int w = 0; !rc && w < 2; ++w) rc = b.launch(x, y, sd, ed, koff, qoff, yq, ypp, nullptr, s);
        if (rc) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; !rc && r < reps; ++r) rc = b.launch(x, y, sd, ed, koff, qoff, yq, ypp, nullptr, s);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) rc = SOLVE_E_DEVICE;
        if (rc) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double per = (double)ms / reps;
        if (per < bms) {
            bms = per;
            bt = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!rc) rc = b.retile(bt);
    if (!rc) rc = b.upload(s);
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = SOLVE_E_DEVICE;
    (void)hipStreamDestroy(s);
    if (rc) return rc;
    *best = bt;
    *best_ms = bms;
    if (cache_path) {
        cache[key] = {(double)bt.block, (double)bt.queries_per_tile, (double)bt.grid_per_cu, (double)bt.fused, bms};
        write_cache(cache_path, cache);
    }
    return SOLVE_OK;
}

extern "C" int spline_plan_destroy(spline_plan* p) {
    if (!p) return SOLVE_E_ARG;
    DeviceGuard g(p->batch.device());
    (void)hipDeviceSynchronize();
    delete p;
    return SOLVE_OK;
}
