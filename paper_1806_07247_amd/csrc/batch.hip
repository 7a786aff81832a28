// Batched tprod and prox_tnn over many tensors of uneven sizes.
//
// A plan lists, per stage of the slice pipeline, every unit of work of every
// tensor: 64 tubes for the transforms, one output tile of one Fourier slice
// for the slice products, one Fourier slice for the SVD and the shrinkage.
// Each stage is one launch of a persistent kernel whose workgroups walk the
// unit list (unit u, u + grid, ...), so a whole batch costs a handful of
// launches whatever the number of tensors:
//   tprod:    forward transforms of all A and B, slice products, inverse transforms
//   prox_tnn: forward transforms, one-sided Jacobi, shrinkage (with the
//             per-tensor tau), the two SVT products, inverse transforms
// The descriptor tables live at the start of the caller's workspace and are
// written once by tp_batch_bind; tp_batch_run then only enqueues kernels, so
// it can be captured into a HIP graph and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "tp_internal.h"

struct tp_batch {
    int op, count, flags;
    tp_batch_opts opts;
    std::vector<tp_batch_item> items;
    // host copies of the tables, uploaded by bind
    std::vector<tp::FftUnit> fwd, inv;
    std::vector<tp::CgemmArgs> g1, g2;
    std::vector<tp::GemmUnit> u1, u2;
    std::vector<tp::JacobiArgs> jac;
    std::vector<tp::ShrinkItem> shr;
    std::vector<tp::SliceUnit> ju, su;
    // Jacobi units in classes of LDS footprint (largest class first), each
    // launched with its own LDS size, so that small slices share a CU
    struct JClass {
        int start, count, max_r, max_p, grid;
    };
    std::vector<JClass> jcls;
    // byte offsets of the tables and the planes in the workspace
    size_t off_fwd = 0, off_inv = 0, off_g1 = 0, off_g2 = 0, off_u1 = 0, off_u2 = 0, off_jac = 0, off_shr = 0,
           off_ju = 0, off_su = 0, tables_end = 0, total = 0;
    std::vector<size_t> off_plane;  // per item: first plane byte offset
    int max_n3 = 0, max_r = 0, max_p = 0, tile = 0;
    int grid_fft = 0, grid_gemm = 0, grid_jac = 0;
    double fwd_bytes = 0, inv_bytes = 0, g1_flops = 0, g1_bytes = 0, g2_flops = 0, g2_bytes = 0;
    char* ws = nullptr;  // bound workspace
    bool bound = false;
    // the Jacobi classes after the first run on side streams, forked from and
    // joined back to the run's stream with events (graph-capturable); made
    // by bind, default priority
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;  // [0]: fork, [1 + i]: join of side stream i
    ~tp_batch()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        for (hipStream_t x : side) (void)hipStreamDestroy(x);
    }
};

namespace {

constexpr int kMaxProxDim = 128;  // slices of the batched prox stay in LDS

size_t al(size_t v) { return tp::align_up(v); }

// the device address of plan table `off` once bound
template <class T>
T* dev(const tp_batch* p, size_t off)
{
    return reinterpret_cast<T*>(p->ws + off);
}

void add_fft_units(std::vector<tp::FftUnit>& out, const float* src, float* re, float* im, float* dst,
                   long long ntubes, int n3)
{
    for (long long b = 0; b < ntubes; b += 64) {
        tp::FftUnit u;
        u.src = src;
        u.re = re;
        u.im = im;
        u.dst = dst;
        u.ntubes = ntubes;
        u.base = b;
        u.n3 = n3;
        u.nt = (int)std::min<long long>(64, ntubes - b);
        out.push_back(u);
    }
}

// product flops and algorithmic bytes of one item's slice product
void gemm_work(const tp::CgemmArgs& a, double& flops, double& bytes)
{
    const int nreal = (a.real_first ? 1 : 0) + (a.real_last && a.nslices > 1 ? 1 : 0);
    const double mnk = (double)a.m * a.n * a.k, el = (double)a.m * a.k + (double)a.k * a.n + (double)a.m * a.n;
    flops += mnk * (8.0 * (a.nslices - nreal) + 2.0 * nreal);
    bytes += el * (8.0 * (a.nslices - nreal) + 4.0 * nreal);
}

void add_gemm_units(std::vector<tp::GemmUnit>& out, int item, const tp::CgemmArgs& a, int op, int tile)
{
    for (int s = 0; s < a.nslices; ++s)
        for (int m0 = 0; m0 < a.m; m0 += tile)
            for (int n0 = 0; n0 < a.n; n0 += tile) out.push_back(tp::GemmUnit{item, s, m0, n0, op});
}

// planes of one item, carved from `off` (bytes, relative to the workspace)
struct Carve {
    size_t off;
    float* base;  // null while sizing
    float* take(size_t count)
    {
        float* p = base ? reinterpret_cast<float*>(reinterpret_cast<char*>(base) + off) : nullptr;
        off += al(count * sizeof(float));
        return p;
    }
};

int plan_layout(tp_batch* p, char* ws)
{
    p->fwd.clear();
    p->inv.clear();
    p->g1.clear();
    p->g2.clear();
    p->u1.clear();
    p->u2.clear();
    p->jac.clear();
    p->shr.clear();
    p->ju.clear();
    p->su.clear();
    p->fwd_bytes = p->inv_bytes = p->g1_flops = p->g1_bytes = p->g2_flops = p->g2_bytes = 0;
    const int tile = tp::batch_tile(p->tile);
    // pass 1: the number of units fixes the table sizes; pass 2 (ws given) the pointers
    size_t cursor = p->tables_end;
    for (int i = 0; i < p->count; ++i) {
        const tp_batch_item& it = p->items[i];
        const int n1 = it.n1, n2 = it.n2, l = it.l, n3 = it.n3, h = tp::half_slices(n3);
        const int rl = (n3 % 2 == 0 && h > 1) ? 1 : 0;
        Carve c{cursor, ws ? reinterpret_cast<float*>(ws) : nullptr};
        const long long mn = (long long)n1 * n2;
        if (p->op == TP_BATCH_TPROD) {
            float* ar = c.take(h * mn);
            float* ai = c.take(h * mn);
            float* br = c.take((size_t)h * n2 * l);
            float* bi = c.take((size_t)h * n2 * l);
            float* cr = c.take((size_t)h * n1 * l);
            float* ci = c.take((size_t)h * n1 * l);
            add_fft_units(p->fwd, it.A, ar, ai, nullptr, mn, n3);
            add_fft_units(p->fwd, it.B, br, bi, nullptr, (long long)n2 * l, n3);
            add_fft_units(p->inv, nullptr, cr, ci, it.C, (long long)n1 * l, n3);
            p->fwd_bytes += (double)(mn + (long long)n2 * l) * (4.0 * n3 + 8.0 * h);
            p->inv_bytes += (double)n1 * l * (4.0 * n3 + 8.0 * h);
            tp::CgemmArgs g{};
            g.ar = ar; g.ai = ai; g.lda = n2; g.sa = mn;
            g.br = br; g.bi = bi; g.ldb = l; g.sb = (long long)n2 * l;
            g.cr = cr; g.ci = ci; g.ldc = l; g.sc = (long long)n1 * l;
            g.m = n1; g.n = l; g.k = n2;
            g.nslices = h; g.real_first = 1; g.real_last = rl;
            add_gemm_units(p->u1, (int)p->g1.size(), g, tp::GEMM_NN, tile);
            gemm_work(g, p->g1_flops, p->g1_bytes);
            p->g1.push_back(g);
        } else {
            const bool tr = n1 < n2;
            const int R = tr ? n2 : n1, P = tr ? n1 : n2;
            float* yr = c.take(h * mn);
            float* yi = c.take(h * mn);
            float* wr = c.take(h * mn);
            float* wi = c.take(h * mn);
            float* tr_ = c.take((size_t)h * P * P);
            float* ti = c.take((size_t)h * P * P);
            double* sig = reinterpret_cast<double*>(c.take((size_t)h * P * 2));
            add_fft_units(p->fwd, it.A, yr, yi, nullptr, mn, n3);
            add_fft_units(p->inv, nullptr, yr, yi, it.C, mn, n3);
            p->fwd_bytes += (double)mn * (4.0 * n3 + 8.0 * h);
            p->inv_bytes += (double)mn * (4.0 * n3 + 8.0 * h);
            tp::JacobiArgs j{};
            j.yr = yr; j.yi = yi; j.wr = wr; j.wi = wi; j.sigma = sig;
            j.m = n1; j.n = n2; j.nslices = h;
            j.max_sweeps = p->opts.max_sweeps > 0 ? p->opts.max_sweeps : tp::param(TP_PARAM_JACOBI_SWEEPS);
            j.transpose = tr ? 1 : 0;
            j.tol = tp::jacobi_tol(R);
            const int ji = (int)p->jac.size();
            p->jac.push_back(j);
            for (int s = 0; s < h; ++s) p->ju.push_back(tp::SliceUnit{ji, s});
            tp::ShrinkItem sh{};
            sh.sigma = sig; sh.wr = wr; sh.wi = wi; sh.R = R; sh.P = P; sh.h = h;
            sh.rel = (p->flags & TP_BATCH_TAU_REL) ? 1 : 0;
            sh.tau = it.tau;
            sh.keep = it.rank;
            sh.tau_out = it.tau_used;
            p->shr.push_back(sh);
            for (int s = 0; s < h; ++s) p->su.push_back(tp::SliceUnit{ji, s});
            tp::CgemmArgs a{}, b{};
            a.nslices = b.nslices = h;
            a.real_first = b.real_first = 1;
            a.real_last = b.real_last = rl;
            int op1, op2;
            if (!tr) {  // T = What^* Ybar (n x n), W = What T
                a.ar = wr; a.ai = wi; a.lda = n2; a.sa = mn;
                a.br = yr; a.bi = yi; a.ldb = n2; a.sb = mn;
                a.cr = tr_; a.ci = ti; a.ldc = P; a.sc = (long long)P * P;
                a.m = n2; a.n = n2; a.k = n1;
                op1 = tp::GEMM_CN;
                b.ar = wr; b.ai = wi; b.lda = n2; b.sa = mn;
                b.br = tr_; b.bi = ti; b.ldb = P; b.sb = (long long)P * P;
                b.cr = yr; b.ci = yi; b.ldc = n2; b.sc = mn;
                b.m = n1; b.n = n2; b.k = n2;
                op2 = tp::GEMM_NN;
            } else {  // T = Ybar Bhat (m x m), W = T Bhat^*
                a.ar = yr; a.ai = yi; a.lda = n2; a.sa = mn;
                a.br = wr; a.bi = wi; a.ldb = n1; a.sb = mn;
                a.cr = tr_; a.ci = ti; a.ldc = P; a.sc = (long long)P * P;
                a.m = n1; a.n = n1; a.k = n2;
                op1 = tp::GEMM_NN;
                b.ar = tr_; b.ai = ti; b.lda = P; b.sa = (long long)P * P;
                b.br = wr; b.bi = wi; b.ldb = n1; b.sb = mn;
                b.cr = yr; b.ci = yi; b.ldc = n2; b.sc = mn;
                b.m = n1; b.n = n2; b.k = n1;
                op2 = tp::GEMM_NC;
            }
            add_gemm_units(p->u1, (int)p->g1.size(), a, op1, tile);
            add_gemm_units(p->u2, (int)p->g2.size(), b, op2, tile);
            gemm_work(a, p->g1_flops, p->g1_bytes);
            gemm_work(b, p->g2_flops, p->g2_bytes);
            p->g1.push_back(a);
            p->g2.push_back(b);
        }
        cursor = c.off;
    }
    // heavy units first (the grid walks the lists in order)
    auto gemm_cost = [&](const std::vector<tp::CgemmArgs>& g) {
        return [&g](const tp::GemmUnit& x, const tp::GemmUnit& y) { return g[x.item].k > g[y.item].k; };
    };
    std::stable_sort(p->u1.begin(), p->u1.end(), gemm_cost(p->g1));
    std::stable_sort(p->u2.begin(), p->u2.end(), gemm_cost(p->g2));
    // Jacobi units: by LDS class (largest first), then by cost within a class
    auto jclass = [&](const tp::JacobiArgs& a) {
        const size_t b = (size_t)a.m * a.n * sizeof(float2);
        return b <= 16 * 1024 ? 0 : (b <= 32 * 1024 ? 1 : (b <= 64 * 1024 ? 2 : 3));
    };
    std::stable_sort(p->ju.begin(), p->ju.end(), [&](const tp::SliceUnit& x, const tp::SliceUnit& y) {
        const tp::JacobiArgs &a = p->jac[x.item], &b = p->jac[y.item];
        const int ka = jclass(a), kb = jclass(b);
        if (ka != kb) return ka > kb;
        const double ca = (double)a.m * a.n * std::min(a.m, a.n), cb = (double)b.m * b.n * std::min(b.m, b.n);
        return ca > cb;
    });
    p->jcls.clear();
    for (int u = 0; u < (int)p->ju.size(); ++u) {
        const tp::JacobiArgs& a = p->jac[p->ju[u].item];
        const int k = jclass(a);
        if (p->jcls.empty() || jclass(p->jac[p->ju[p->jcls.back().start].item]) != k)
            p->jcls.push_back(tp_batch::JClass{u, 0, 0, 0, 0});
        tp_batch::JClass& c = p->jcls.back();
        ++c.count;
        c.max_r = std::max(c.max_r, std::max(a.m, a.n));
        c.max_p = std::max(c.max_p, std::min(a.m, a.n));
    }
    for (tp_batch::JClass& c : p->jcls) {
        const size_t lds = tp::jacobi_batch_lds(c.max_r, c.max_p);
        const int per_cu = std::max(1, std::min(8, (int)((160 * 1024 - 1024) / std::max<size_t>(lds, 1))));
        c.grid = p->opts.grid_jacobi > 0 ? p->opts.grid_jacobi : 256 * per_cu;
    }
    return (int)(cursor - p->tables_end);
}

template <class T>
size_t table(size_t& cur, const std::vector<T>& v)
{
    const size_t off = cur;
    cur += al(std::max<size_t>(v.size(), 1) * sizeof(T));
    return off;
}

int clamp_grid(int requested, int dflt) { return requested > 0 ? requested : dflt; }

}  // namespace

extern "C" {

int tp_batch_create(tp_batch** out, int op, const tp_batch_item* items, int count, int flags,
                    const tp_batch_opts* opts)
{
    if (!out) return TP_ERR_ARG;
    *out = nullptr;
    if ((op != TP_BATCH_TPROD && op != TP_BATCH_PROX) || !items || count <= 0 || (flags & ~TP_BATCH_TAU_REL))
        return TP_ERR_ARG;
    if (op == TP_BATCH_TPROD && (flags & TP_BATCH_TAU_REL)) return TP_ERR_ARG;
    tp_batch_opts o{};
    if (opts) o = *opts;
    if (o.tile < 0 || o.tile > 2 || o.grid_fft < 0 || o.grid_gemm < 0 || o.grid_jacobi < 0 || o.max_sweeps < 0)
        return TP_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        const tp_batch_item& it = items[i];
        if (!it.A || !it.C) return TP_ERR_ARG;
        if (it.n1 <= 0 || it.n2 <= 0 || it.n3 <= 0 || it.n3 > tp::kBatchMaxN3) return TP_ERR_SHAPE;
        if (op == TP_BATCH_TPROD) {
            if (!it.B) return TP_ERR_ARG;
            if (it.l <= 0 || it.n1 > 65536 || it.n2 > 65536 || it.l > 65536) return TP_ERR_SHAPE;
        } else {
            if (it.n1 > kMaxProxDim || it.n2 > kMaxProxDim) return TP_ERR_SHAPE;
            if (!(it.tau >= 0.0f) || std::isinf(it.tau)) return TP_ERR_ARG;
        }
    }
    tp_batch* p = new (std::nothrow) tp_batch();
    if (!p) return TP_ERR_ARG;
    p->op = op;
    p->count = count;
    p->flags = flags;
    p->opts = o;
    p->items.assign(items, items + count);
    for (const tp_batch_item& it : p->items) {
        p->max_n3 = std::max(p->max_n3, it.n3);
        p->max_r = std::max(p->max_r, std::max(it.n1, it.n2));
        p->max_p = std::max(p->max_p, std::min(it.n1, it.n2));
    }
    // tile: tuned, else 32 x 32 unless most products are large
    if (o.tile > 0) {
        p->tile = o.tile - 1;
    } else {
        double small = 0, all = 0;
        for (const tp_batch_item& it : p->items) {
            const double m = it.n1, n = (op == TP_BATCH_TPROD) ? it.l : it.n2;
            all += 1;
            small += (m <= 64 || n <= 64) ? 1 : 0;
        }
        p->tile = (small >= 0.5 * all) ? 0 : 1;
    }
    // sizing pass: unit counts, then the table offsets and the plane bytes
    p->tables_end = 0;
    plan_layout(p, nullptr);
    size_t cur = 0;
    p->off_fwd = table(cur, p->fwd);
    p->off_inv = table(cur, p->inv);
    p->off_g1 = table(cur, p->g1);
    p->off_g2 = table(cur, p->g2);
    p->off_u1 = table(cur, p->u1);
    p->off_u2 = table(cur, p->u2);
    p->off_jac = table(cur, p->jac);
    p->off_shr = table(cur, p->shr);
    p->off_ju = table(cur, p->ju);
    p->off_su = table(cur, p->su);
    p->tables_end = cur;
    p->total = cur + (size_t)plan_layout(p, nullptr);
    p->grid_fft = clamp_grid(o.grid_fft, 256 * 16);
    p->grid_gemm = clamp_grid(o.grid_gemm, 256 * (p->tile == 0 ? 8 : 4));
    const size_t lds = tp::jacobi_batch_lds(p->max_r, p->max_p);
    const int per_cu = std::max(1, (int)((160 * 1024 - 1024) / std::max<size_t>(lds, 1)));
    p->grid_jac = clamp_grid(o.grid_jacobi, 256 * std::min(per_cu, 8));
    *out = p;
    return TP_OK;
}

size_t tp_batch_workspace_size(const tp_batch* p) { return p ? p->total : 0; }

int tp_batch_bind(tp_batch* p, void* workspace, size_t workspace_bytes, void* stream)
{
    if (!p || !workspace) return TP_ERR_ARG;
    if (workspace_bytes < p->total) return TP_ERR_WORKSPACE;
    p->ws = static_cast<char*>(workspace);
    plan_layout(p, p->ws);  // the same layout with device pointers
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(p->ws + off, src, bytes, hipMemcpyHostToDevice, s);
    };
#define TP_UP(off, v) TP_TRY(up(off, v.data(), v.size() * sizeof(v[0])))
    TP_UP(p->off_fwd, p->fwd);
    TP_UP(p->off_inv, p->inv);
    TP_UP(p->off_g1, p->g1);
    TP_UP(p->off_g2, p->g2);
    TP_UP(p->off_u1, p->u1);
    TP_UP(p->off_u2, p->u2);
    TP_UP(p->off_jac, p->jac);
    TP_UP(p->off_shr, p->shr);
    TP_UP(p->off_ju, p->ju);
    TP_UP(p->off_su, p->su);
#undef TP_UP
    if (p->op != TP_BATCH_TPROD && p->jcls.size() > 1 && p->side.empty()) {
        for (size_t i = 1; i < p->jcls.size(); ++i) {
            hipStream_t x;
            TP_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
            p->side.push_back(x);
        }
        for (size_t i = 0; i < p->jcls.size(); ++i) {
            hipEvent_t e;
            TP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            p->ev.push_back(e);
        }
    }
    TP_TRY(hipStreamSynchronize(s));
    p->bound = true;
    return TP_OK;
}

int tp_batch_run(const tp_batch* p, void* stream)
{
    if (!p || !p->bound) return TP_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nf = (int)p->fwd.size(), ni = (int)p->inv.size();
    TP_LAUNCH(tp::K_RFFT, s,
              (tp::trace_work(0.0, p->fwd_bytes),
               tp::launch_fft_batch(dev<tp::FftUnit>(p, p->off_fwd), nf, 0, p->max_n3, p->grid_fft, s)));
    if (p->op == TP_BATCH_TPROD) {
        TP_LAUNCH(tp::K_CGEMM, s,
                  tp::launch_cgemm_batch(dev<tp::CgemmArgs>(p, p->off_g1), dev<tp::GemmUnit>(p, p->off_u1),
                                         (int)p->u1.size(), p->tile, p->grid_gemm, p->g1_flops, p->g1_bytes, s));
    } else {
        // the classes touch disjoint slices: the first on the run's stream,
        // the others at the same time on the side streams
        const size_t nside = p->side.size();
        if (nside) TP_TRY(hipEventRecord(p->ev[0], s));
        for (size_t i = 0; i < p->jcls.size(); ++i) {
            const tp_batch::JClass& c = p->jcls[i];
            hipStream_t cs = (i == 0 || nside == 0) ? s : p->side[i - 1];
            if (cs != s) TP_TRY(hipStreamWaitEvent(cs, p->ev[0], 0));
            TP_LAUNCH(tp::K_JACOBI, cs,
                      tp::launch_jacobi_batch(dev<tp::JacobiArgs>(p, p->off_jac),
                                              dev<tp::SliceUnit>(p, p->off_ju) + c.start, c.count, c.max_r, c.max_p,
                                              c.grid, cs));
            if (cs != s) TP_TRY(hipEventRecord(p->ev[i], cs));
        }
        for (size_t i = 1; nside && i < p->jcls.size(); ++i) TP_TRY(hipStreamWaitEvent(s, p->ev[i], 0));
        TP_LAUNCH(tp::K_SHRINK, s,
                  tp::launch_shrink_batch(dev<tp::ShrinkItem>(p, p->off_shr), dev<tp::SliceUnit>(p, p->off_su),
                                          (int)p->su.size(), p->grid_jac, s));
        TP_LAUNCH(tp::K_CGEMM, s,
                  tp::launch_cgemm_batch(dev<tp::CgemmArgs>(p, p->off_g1), dev<tp::GemmUnit>(p, p->off_u1),
                                         (int)p->u1.size(), p->tile, p->grid_gemm, p->g1_flops, p->g1_bytes, s));
        TP_LAUNCH(tp::K_CGEMM, s,
                  tp::launch_cgemm_batch(dev<tp::CgemmArgs>(p, p->off_g2), dev<tp::GemmUnit>(p, p->off_u2),
                                         (int)p->u2.size(), p->tile, p->grid_gemm, p->g2_flops, p->g2_bytes, s));
    }
    TP_LAUNCH(tp::K_IRFFT, s,
              (tp::trace_work(0.0, p->inv_bytes),
               tp::launch_fft_batch(dev<tp::FftUnit>(p, p->off_inv), ni, 1, p->max_n3, p->grid_fft, s)));
    return TP_OK;
}

int tp_batch_stats(const tp_batch* p, tp_batch_stats_t* st)
{
    if (!p || !st) return TP_ERR_ARG;
    st->fft_units = (int)(p->fwd.size() + p->inv.size());
    st->gemm_units = (int)(p->u1.size() + p->u2.size());
    st->slice_units = (int)p->ju.size();
    st->tile = tp::batch_tile(p->tile);
    st->grid_fft = p->grid_fft;
    st->grid_gemm = p->grid_gemm;
    st->grid_jacobi = p->grid_jac;
    st->gemm_flops = p->g1_flops + p->g2_flops;
    st->fft_bytes = p->fwd_bytes + p->inv_bytes;
    return TP_OK;
}

int tp_batch_destroy(tp_batch* p)
{
    delete p;
    return TP_OK;
}

}  // extern "C"
