// Host-side runtime services: tunable launch parameters and stage timing
// (HIP events recorded around every kernel the entry points enqueue, while
// enabled).  Nothing here runs on the device.
#include <algorithm>
#include <mutex>
#include <vector>

#include "tp_internal.h"

namespace tp {
namespace {

// a slice product whose gate or sizes live on the device (resolved when collected)
struct DynWork {
    bool on;
    const int *gate, *m, *n, *k;
    int hm, hn, hk, nslices, nreal;
};

struct Rec {
    hipEvent_t a, b;
    int id;
    double flops, bytes;
    DynWork dyn;
};

// work reported inside the innermost open scope of this thread
thread_local double t_flops = 0.0, t_bytes = 0.0;
thread_local DynWork t_dyn{};

int read_dev(const int* p, int dflt)
{
    if (!p) return dflt;
    int v = dflt;
    if (hipMemcpy(&v, p, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return dflt;
    return v;
}

std::mutex g_mu;
bool g_on = false;
std::vector<hipEvent_t> g_pool;
std::vector<Rec> g_recs;

hipEvent_t take_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

const char* const kNames[] = {"rfft",    "irfft",   "cgemm",  "jacobi",     "shrink", "tnn_reduce", "tsvd_finish",
                              "features", "predict", "sketch", "cholqr", "rsvd_check", "gather",     "mlp",
                              "accuracy", "tensor_op", "trpca"};

}  // namespace

TraceScope::TraceScope(hipStream_t s, int id) : stream_(s), id_(id), start_(nullptr)
{
    t_flops = 0.0;
    t_bytes = 0.0;
    t_dyn.on = false;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    start_ = take_event();
    if (start_) hipEventRecord(static_cast<hipEvent_t>(start_), s);
}

TraceScope::~TraceScope()
{
    if (!start_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t b = take_event();
    if (!b) return;
    hipEventRecord(b, stream_);
    g_recs.push_back(Rec{static_cast<hipEvent_t>(start_), b, id_, t_flops, t_bytes, t_dyn});
}

void trace_work(double flops, double bytes)
{
    t_flops += flops;
    t_bytes += bytes;
}

void trace_gemm_dyn(const int* gate, const int* m, const int* n, const int* k, int hm, int hn, int hk, int nslices,
                    int nreal)
{
    t_dyn = DynWork{true, gate, m, n, k, hm, hn, hk, nslices, nreal};
}

namespace {
int g_params[TP_PARAM_COUNT] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
const int kDefaults[TP_PARAM_COUNT] = {0, 0, 128, 30, 0, 8, 1, 0, 0, 0, 2, 0, 0};
}  // namespace

int param(int key)
{
    if (key < 0 || key >= TP_PARAM_COUNT) return 0;
    const int v = __atomic_load_n(&g_params[key], __ATOMIC_RELAXED);
    return v > 0 ? v : kDefaults[key];
}

}  // namespace tp

extern "C" {

int tp_set_param(int key, int value)
{
    if (key < 0 || key >= TP_PARAM_COUNT || value < 0) return TP_ERR_ARG;
    __atomic_store_n(&tp::g_params[key], value, __ATOMIC_RELAXED);
    return TP_OK;
}

int tp_get_param(int key)
{
    if (key < 0 || key >= TP_PARAM_COUNT) return -1;
    return tp::param(key);
}

int tp_trace_enable(int enable)
{
    std::lock_guard<std::mutex> lk(tp::g_mu);
    tp::g_on = enable != 0;
    return TP_OK;
}

int tp_trace_collect(int* kernel_ids, float* ms, int capacity)
{
    return tp_trace_collect_work(kernel_ids, ms, nullptr, nullptr, capacity);
}

int tp_trace_collect_work(int* kernel_ids, float* ms, double* flops, double* bytes, int capacity)
{
    std::lock_guard<std::mutex> lk(tp::g_mu);
    int n = 0;
    for (const tp::Rec& r : tp::g_recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return TP_ERR_HIP;
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return TP_ERR_HIP;
        double fl = r.flops, by = r.bytes;
        if (r.dyn.on) {  // the gate and live sizes as they are in device memory now
            const tp::DynWork& d = r.dyn;
            const bool run = tp::read_dev(d.gate, 1) != 0;
            const double m = std::min(d.hm, tp::read_dev(d.m, d.hm)), nn = std::min(d.hn, tp::read_dev(d.n, d.hn)),
                         k = std::min(d.hk, tp::read_dev(d.k, d.hk));
            const int cplx = d.nslices - d.nreal;
            fl = run ? m * nn * k * (8.0 * cplx + 2.0 * d.nreal) : 0.0;
            by = run ? (m * k + k * nn + m * nn) * (8.0 * cplx + 4.0 * d.nreal) : 0.0;
        }
        if (n < capacity) {
            if (kernel_ids) kernel_ids[n] = r.id;
            if (ms) ms[n] = t;
            if (flops) flops[n] = fl;
            if (bytes) bytes[n] = by;
        }
        ++n;
        tp::g_pool.push_back(r.a);
        tp::g_pool.push_back(r.b);
    }
    tp::g_recs.clear();
    return n;
}

const char* tp_kernel_name(int id)
{
    if (id < 0 || id >= (int)(sizeof(tp::kNames) / sizeof(tp::kNames[0]))) return "unknown";
    return tp::kNames[id];
}

}  // extern "C"
