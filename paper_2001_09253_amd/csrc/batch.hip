// Batched spline path: persistent fused kernel, its two-launch form, hipGraph
// capture and the autotuner (C ABI: spline_plan_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include "batch.hpp"
#include "spline_kernels.hpp"
#include "spline_solve.h"

namespace spl {

constexpr int kSpinLimit = 1 << 25;  // ~ seconds of s_sleep before a tile gives up waiting
constexpr int kBatchWin = kBatchWindow;  // staged knot window of an evaluate slice

template <int BLOCK, int QPT>
struct FusedSmem {
    static constexpr int kNW = BLOCK / kWave;
    static constexpr int kCHB = SOLVE_MAX_N_BATCH / BLOCK;  // rows per lane of a whole-group build
    static constexpr int kBuildDoubles =
        (BLOCK * kCHB > kNW * kWaveBuildMaxN) ? BLOCK * kCHB : kNW * kWaveBuildMaxN;
    union {
        UniSmem<BLOCK, QPT, kBatchWin> ev;
        double build[kBuildDoubles];
    };
    Fwd lds_f[kNW];
    Bwd lds_b[kNW];
    int item;
};

// Build one work item.  Every lane of the workgroup calls this.
template <int BLOCK, int QPT>
__device__ void run_build_item(const BatchDevArgs& a, const BuildItem& bi, FusedSmem<BLOCK, QPT>& sm,
                               bool signal) {
    using S = FusedSmem<BLOCK, QPT>;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    if (bi.kind == kItemWhole) {
        const int i = bi.inst[0];
        const int64_t o = a.koff[i];
        const int n = (int)(a.koff[i + 1] - o);
        build_group<BLOCK, S::kCHB, false>(a.x + o, a.y + o, n, a.sd[i], a.ed[i], a.ypp + o,
                                           a.status ? a.status + i : nullptr, sm.build, sm.lds_f, sm.lds_b, tid);
    } else {
        const int i = wid < kItemLanes ? bi.inst[wid] : -1;
        if (i >= 0) {
            const int64_t o = a.koff[i];
            const int n = (int)(a.koff[i + 1] - o);
            build_group<kWave, kWaveBuildMaxN / kWave, true>(a.x + o, a.y + o, n, a.sd[i], a.ed[i], a.ypp + o,
                                                             a.status ? a.status + i : nullptr,
                                                             sm.build + wid * kWaveBuildMaxN, nullptr, nullptr,
                                                             lane);
        }
    }
    if (signal) {
        // one release for the whole item, then its curves' ready flags
        __syncthreads();
        if (tid == 0) release_fence_agent();
        __syncthreads();
        if (tid < kItemLanes) {
            const int i = bi.kind == kItemWhole ? (tid == 0 ? bi.inst[0] : -1) : bi.inst[tid];
            if (i >= 0) __hip_atomic_store(&a.ready[i], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int BLOCK, int QPT>
__device__ void run_tile(const BatchDevArgs& a, const TileItem& ti, FusedSmem<BLOCK, QPT>& sm) {
    const int i = ti.inst;
    const int64_t o = a.koff[i];
    const int64_t n = a.koff[i + 1] - o;
    const int64_t qo = a.qoff[i];
    const int64_t m = a.qoff[i + 1] - qo;
    eval_uniform_range<BLOCK, QPT, kBatchWin, kModeValue, false>(a.x + o, a.y + o, a.ypp + o, n, m, ti.k0, ti.k1,
                                                                 a.yq + qo, sm.ev, threadIdx.x);
}

template <int BLOCK, int QPT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void fused_kernel(BatchDevArgs a) {
    __shared__ FusedSmem<BLOCK, QPT> sm;
    const int tid = threadIdx.x;
    // Phase 1: claim build items until none are left.
    for (;;) {
        if (tid == 0) sm.item = atomicAdd(&a.counters[0], 1);
        __syncthreads();
        const int it = sm.item;
        __syncthreads();
        if (it >= a.n_items) break;
        run_build_item<BLOCK, QPT>(a, a.items[it], sm, true);
        __syncthreads();
    }
    // Phase 2: evaluate tiles with a grid stride, each after its curve is ready.
    for (int t = blockIdx.x; t < a.n_tiles; t += gridDim.x) {
        const TileItem ti = a.tiles[t];
        if (tid == 0) (void)wait_flag_at_least<2>(&a.ready[ti.inst], 1, kSpinLimit, &a.counters[1]);
        __syncthreads();
        run_tile<BLOCK, QPT>(a, ti, sm);
        __syncthreads();
    }
}

// Two-launch form: one workgroup per build item, then one per tile.
template <int BLOCK, int QPT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void build_items_kernel(BatchDevArgs a) {
    __shared__ FusedSmem<BLOCK, QPT> sm;
    run_build_item<BLOCK, QPT>(a, a.items[blockIdx.x], sm, false);
}

template <int BLOCK, int QPT>
__global__ __launch_bounds__(BLOCK) void eval_tiles_kernel(BatchDevArgs a) {
    __shared__ FusedSmem<BLOCK, QPT> sm;
    run_tile<BLOCK, QPT>(a, a.tiles[blockIdx.x], sm);
}

// Clears the claim counter, the timeout flag and the ready flags (a kernel, so
// that it can sit in a captured graph).
__global__ void reset_kernel(int32_t* counters, int32_t* ready, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 4) counters[i] = 0;
    for (int64_t j = i; j < count; j += (int64_t)gridDim.x * blockDim.x) ready[j] = 0;
}

template <int BLOCK, int QPT>
static int launch_variant(const BatchDevArgs& a, int fused, int grid, int64_t count, hipStream_t s) {
    if (fused) {
        const int rb = 256;
        const int rg = (int)std::min<int64_t>(1024, (count + rb - 1) / rb + 1);
        reset_kernel<<<rg, rb, 0, s>>>(a.counters, a.ready, count);
        fused_kernel<BLOCK, QPT><<<grid, BLOCK, 0, s>>>(a);
    } else {
        if (a.n_items > 0) build_items_kernel<BLOCK, QPT><<<a.n_items, BLOCK, 0, s>>>(a);
        if (a.n_tiles > 0) eval_tiles_kernel<BLOCK, QPT><<<a.n_tiles, BLOCK, 0, s>>>(a);
    }
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

spline_tuning default_tuning() {
    spline_tuning t;
    t.block = 256;
    t.queries_per_tile = 8192;
    t.grid_per_cu = 4;
    t.fused = 0;
    return t;
}

bool valid_tuning(const spline_tuning& t) {
    return (t.block == 256 || t.block == 512) && t.queries_per_tile >= t.block &&
           t.queries_per_tile <= (1 << 24) && t.grid_per_cu >= 1 && t.grid_per_cu <= 8 &&
           (t.fused == 0 || t.fused == 1);
}

Batch::~Batch() {
    hipFree(d_items_);
    hipFree(d_tiles_);
    hipFree(d_counters_);
}

int Batch::ensure(void** p, size_t* cap, size_t bytes) {
    if (bytes <= *cap && *p) return SOLVE_OK;
    size_t want = std::max<size_t>(bytes, 256);
    want = std::max(want, *cap + *cap / 2);
    if (*p) hipFree(*p);
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
    const int nw = tuning_.block / kWave;
    items_.clear();
    tiles_.clear();
    // Larger curves first: a whole workgroup each, claimed early.
    for (int64_t i = 0; i < count_; ++i) {
        if (n_[i] > kWaveBuildMaxN) {
            BuildItem b;
            b.kind = kItemWhole;
            for (int w = 0; w < kItemLanes; ++w) b.inst[w] = -1;
            b.inst[0] = (int32_t)i;
            items_.push_back(b);
        }
    }
    BuildItem cur;
    int fill = 0;
    for (int64_t i = 0; i < count_; ++i) {
        if (n_[i] > kWaveBuildMaxN) continue;
        if (fill == 0) {
            cur.kind = kItemPacked;
            for (int w = 0; w < kItemLanes; ++w) cur.inst[w] = -1;
        }
        cur.inst[fill++] = (int32_t)i;
        if (fill == nw) {
            items_.push_back(cur);
            fill = 0;
        }
    }
    if (fill) items_.push_back(cur);
    const int64_t cap = tuning_.queries_per_tile;
    for (int64_t i = 0; i < count_; ++i) {
        if (!uniform_[i]) continue;
        // about 0.45 * window intervals per slice keeps the guessed window
        // covering it; a slice is never below one workgroup's worth
        const double per_interval = (double)m_[i] / (double)(n_[i] - 1);
        int64_t sz = (int64_t)(0.45 * kBatchWindow * per_interval);
        sz = std::min<int64_t>(sz, cap);
        sz = std::max<int64_t>(sz, tuning_.block);
        for (int64_t k = 0; k < m_[i]; k += sz)
            tiles_.push_back(TileItem{(int32_t)i, 0, k, std::min<int64_t>(m_[i], k + sz)});
    }
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
    for (int64_t i = 0; i < count; ++i) {
        n_[i] = koff[i + 1] - koff[i];
        m_[i] = qoff[i + 1] - qoff[i];
        if (uniform) uniform_[i] = uniform[i] ? 1 : 0;
        if (n_[i] < 3 || n_[i] > SOLVE_MAX_N_BATCH || m_[i] < (uniform_[i] ? 1 : 0)) return SOLVE_E_SIZE;
    }
    count_ = count;
    total_n_ = koff[count];
    total_m_ = qoff[count];
    tuning_ = t;
    precision_ = precision;
    make_tables();
    if (tiles_.size() > 0x7fffffffULL || items_.size() > 0x7fffffffULL) return SOLVE_E_SIZE;
    if (!num_cu_) {
        if (hipDeviceGetAttribute(&num_cu_, hipDeviceAttributeMultiprocessorCount, device_) != hipSuccess)
            return SOLVE_E_DEVICE;
    }
    int rc = ensure(&d_items_, &cap_items_, items_.size() * sizeof(BuildItem));
    if (!rc) rc = ensure(&d_tiles_, &cap_tiles_, tiles_.size() * sizeof(TileItem));
    if (!rc) rc = ensure(&d_counters_, &cap_counters_, (4 + (size_t)count) * sizeof(int32_t));
    return rc;
}

int Batch::retile(const spline_tuning& t) {
    if (!valid_tuning(t)) return SOLVE_E_ARG;
    tuning_ = t;
    make_tables();
    int rc = ensure(&d_items_, &cap_items_, items_.size() * sizeof(BuildItem));
    if (!rc) rc = ensure(&d_tiles_, &cap_tiles_, tiles_.size() * sizeof(TileItem));
    return rc;
}

int Batch::upload(hipStream_t s) {
    if (!items_.empty() &&
        hipMemcpyAsync(d_items_, items_.data(), items_.size() * sizeof(BuildItem), hipMemcpyHostToDevice, s) !=
            hipSuccess)
        return SOLVE_E_DEVICE;
    if (!tiles_.empty() &&
        hipMemcpyAsync(d_tiles_, tiles_.data(), tiles_.size() * sizeof(TileItem), hipMemcpyHostToDevice, s) !=
            hipSuccess)
        return SOLVE_E_DEVICE;
    return SOLVE_OK;
}

int Batch::upload_staged(hipStream_t s, void* pinned) {
    const size_t bi = items_.size() * sizeof(BuildItem);
    const size_t bt = tiles_.size() * sizeof(TileItem);
    if (bi) std::memcpy(pinned, items_.data(), bi);
    if (bt) std::memcpy((char*)pinned + bi, tiles_.data(), bt);
    if (bi && hipMemcpyAsync(d_items_, pinned, bi, hipMemcpyHostToDevice, s) != hipSuccess) return SOLVE_E_DEVICE;
    if (bt && hipMemcpyAsync(d_tiles_, (char*)pinned + bi, bt, hipMemcpyHostToDevice, s) != hipSuccess)
        return SOLVE_E_DEVICE;
    return SOLVE_OK;
}

int Batch::launch(const double* x, const double* y, const double* sd, const double* ed, const int64_t* koff,
                  const int64_t* qoff, double* yq, double* ypp, int32_t* status, hipStream_t s) {
    if (!x || !y || !sd || !ed || !koff || !qoff || !yq || !ypp) return SOLVE_E_ARG;
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
    a.items = (const BuildItem*)d_items_;
    a.tiles = (const TileItem*)d_tiles_;
    a.counters = (int32_t*)d_counters_;
    a.ready = (int32_t*)d_counters_ + 4;
    a.n_items = (int32_t)items_.size();
    a.n_tiles = (int32_t)tiles_.size();
    a.precision = (int32_t)precision_;
    const int grid = std::max(1, num_cu_ * tuning_.grid_per_cu);
    const int f = tuning_.fused;
    if (tuning_.block == 256) return launch_variant<256, 8>(a, f, grid, count_, s);
    if (tuning_.block == 512) return launch_variant<512, 4>(a, f, grid, count_, s);
    return SOLVE_E_ARG;
}

int32_t Batch::spin_timeout_flag_host() {
    int32_t v = 0;
    if (d_counters_) hipMemcpy(&v, (int32_t*)d_counters_ + 1, sizeof(v), hipMemcpyDeviceToHost);
    return v;
}

}  // namespace spl

using namespace spl;

struct spline_plan {
    Batch batch;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    explicit spline_plan(int dev) : batch(dev) {}
    ~spline_plan() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
    }
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        hipGetDevice(&prev);
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) hipSetDevice(prev);
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
    if (p->exec) { hipGraphExecDestroy(p->exec); p->exec = nullptr; }
    if (p->graph) { hipGraphDestroy(p->graph); p->graph = nullptr; }
    int rc = SOLVE_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = SOLVE_E_DEVICE;
    if (!rc) {
        const int lrc = p->batch.launch(x, y, sd, ed, koff, qoff, yq, ypp, status, s);
        hipGraph_t gr = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &gr);
        if (lrc) rc = lrc;
        else if (e != hipSuccess || !gr) rc = SOLVE_E_DEVICE;
        if (gr && rc) hipGraphDestroy(gr);
        if (!rc) {
            p->graph = gr;
            if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
                p->exec = nullptr;
                rc = SOLVE_E_DEVICE;
            }
        }
    }
    if (cs) hipStreamDestroy(cs);
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
    std::vector<spline_tuning> cands;
    for (int block : {256, 512}) {
        for (int cap : {2048, 4096, 8192, 16384}) {
            for (int gpc : {2, 4, 8}) cands.push_back(spline_tuning{block, cap, gpc, 1});
            cands.push_back(spline_tuning{block, cap, 4, 0});
        }
    }
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return SOLVE_E_DEVICE;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    double bms = 1e300;
    spline_tuning bt = b.tuning();
    int rc = SOLVE_OK;
    for (const auto& t : cands) {
        rc = b.retile(t);
        if (!rc) rc = b.upload(s);
        for (int w = 0; !rc && w < 2; ++w) rc = b.launch(x, y, sd, ed, koff, qoff, yq, ypp, nullptr, s);
        if (rc) break;
        hipEventRecord(e0, s);
        for (int r = 0; !rc && r < reps; ++r) rc = b.launch(x, y, sd, ed, koff, qoff, yq, ypp, nullptr, s);
        hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) rc = SOLVE_E_DEVICE;
        if (rc) break;
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        const double per = (double)ms / reps;
        if (per < bms) {
            bms = per;
            bt = t;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (!rc) rc = b.retile(bt);
    if (!rc) rc = b.upload(s);
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = SOLVE_E_DEVICE;
    hipStreamDestroy(s);
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
    hipDeviceSynchronize();
    delete p;
    return SOLVE_OK;
}
