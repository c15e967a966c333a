// Host runtime of the PIC library: parameter validation, workspace layout, kernel
// dispatch and diagnostics behind the C ABI declared in include/pic.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pic.h"
#include "pic_device.hpp"

using namespace pic;

namespace {

thread_local std::string g_last_error;

constexpr int kDefaultThreads = 256;
constexpr int kDefaultRecords = 4096;
constexpr size_t kAlign = 256;
constexpr size_t kMaxLds = 64 * 1024;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    size_t Ef[2], Bf[2], J1[2], J2[2], cninv, spart, st, rec, total;
};

int threads_of(const pic_params *p) { return p->block_threads ? p->block_threads : kDefaultThreads; }

int records_of(const pic_params *p) { return p->record_capacity ? p->record_capacity : kDefaultRecords; }

int blocks_of(const pic_params *p, int64_t *chunk_out)
{
    const int t = threads_of(p);
    int64_t nb = p->grid_blocks ? p->grid_blocks : std::min<int64_t>((p->n_particles + t - 1) / t, 1024);
    nb = std::max<int64_t>(1, std::min<int64_t>(nb, kMaxGrid));
    // chunks are whole multiples of the batch a workgroup loads at once (4 particles
    // per thread), so only the last workgroup has a ragged tail
    int64_t chunk = (p->n_particles + nb - 1) / nb;
    chunk = (chunk + 4 * t - 1) / (4 * t) * (4 * t);
    nb = (p->n_particles + chunk - 1) / chunk;
    if (chunk_out)
        *chunk_out = chunk;
    return (int)nb;
}

bool is_em(const pic_params *p) { return p->scheme == PIC_EMEC_LI; }

// LDS bytes of the largest kernel of this configuration.
size_t lds_pass_a(const pic_params *p)
{
    // jt | es | bs
    const size_t ng = p->n_cells;
    return is_em(p) ? (3 + 3 + 2) * ng * 8 : 2 * ng * 8;
}

size_t lds_pass_b(const pic_params *p)
{
    // jt | es | bs | eb | bb | e1 | b1 | (EM) Crank-Nicolson scratch
    const size_t ng = p->n_cells;
    return is_em(p) ? (3 + 3 + 2 + 3 + 2 + 3 + 2 + 8) * ng * 8 : 4 * ng * 8;
}

size_t lds_need(const pic_params *p)
{
    return std::max(std::max(lds_pass_a(p), lds_pass_b(p)), (size_t)3 * p->n_cells * 8);
}

Layout layout_of(const pic_params *p)
{
    Layout L;
    const size_t ng = (size_t)p->n_cells;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, kAlign); return at; };
    for (int k = 0; k < 2; ++k) {
        L.Ef[k] = take(3 * ng * 8);
        L.Bf[k] = take(2 * ng * 8);
        L.J1[k] = take(3 * ng * 8);
        L.J2[k] = take(3 * ng * 8);
    }
    L.cninv = take(ng * 8);
    L.spart = take((size_t)blocks_of(p, nullptr) * kNS * 8);
    L.st = take(sizeof(DevState));
    L.rec = take((size_t)records_of(p) * sizeof(DevRecord));
    L.total = o;
    return L;
}

int fail(std::string *where, int code, const char *fmt, ...)
    __attribute__((format(printf, 3, 4)));

int fail(std::string *where, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (where)
        *where = buf;
    g_last_error = buf;
    return code;
}

int validate(const pic_params *p, std::string *err)
{
    if (!p)
        return fail(err, PIC_EINVAL, "params is NULL");
    if (p->abi_version != PIC_ABI_VERSION)
        return fail(err, PIC_EINVAL, "abi_version %d != %d", p->abi_version, PIC_ABI_VERSION);
    if (p->nv != 1 && p->nv != 3)
        return fail(err, PIC_EINVAL, "nv must be 1 or 3 (got %d)", p->nv);
    if (p->scheme < PIC_ESEC2 || p->scheme > PIC_EMEC_LI)
        return fail(err, PIC_EINVAL, "unknown scheme %d", p->scheme);
    if (p->scheme == PIC_EMEC_LI && p->nv != 3)
        return fail(err, PIC_EINVAL, "PIC_EMEC_LI needs nv == 3");
    if (p->shape_order != 1 && p->shape_order != 2)
        return fail(err, PIC_EINVAL, "shape_order must be 1 or 2 (got %d)", p->shape_order);
    if (p->n_particles < 1)
        return fail(err, PIC_EINVAL, "n_particles must be >= 1");
    if (p->n_particles > ((int64_t)1 << 40))
        return fail(err, PIC_EUNSUPPORTED, "n_particles above 2^40");
    if (p->n_cells < 2 * p->shape_order + 1)
        return fail(err, PIC_EINVAL, "n_cells must be >= 2*shape_order+1 (got %d)", p->n_cells);
    if (!(p->length > 0.0) || !std::isfinite(p->length))
        return fail(err, PIC_EINVAL, "length must be finite and > 0");
    if (!(p->dt > 0.0) || !std::isfinite(p->dt))
        return fail(err, PIC_EINVAL, "dt must be finite and > 0");
    if (p->scheme == PIC_EMEC_LI && (!(p->c > 0.0) || !std::isfinite(p->c)))
        return fail(err, PIC_EINVAL, "c must be finite and > 0 for PIC_EMEC_LI");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(p->b_ext[i]))
            return fail(err, PIC_EINVAL, "b_ext must be finite");
    if (p->rebin_every < 0)
        return fail(err, PIC_EINVAL, "rebin_every must be >= 0");
    if (p->rebin_every > 0)
        return fail(err, PIC_EUNSUPPORTED, "rebin_every > 0 is not available in this build");
    if (p->flags & ~(uint32_t)(PIC_F_INIT_GAUSS | PIC_F_TRACK_IDS))
        return fail(err, PIC_EINVAL, "unknown flag bits 0x%x", p->flags);
    if (p->block_threads && (p->block_threads % 64 || p->block_threads < 64 || p->block_threads > 1024))
        return fail(err, PIC_EINVAL, "block_threads must be 0 or a multiple of 64 in [64, 1024]");
    if (p->grid_blocks < 0 || p->grid_blocks > kMaxGrid)
        return fail(err, PIC_EINVAL, "grid_blocks must be in [0, %d]", kMaxGrid);
    if (p->deposit_mode < PIC_DEPOSIT_AUTO || p->deposit_mode > PIC_DEPOSIT_WAVE_REDUCE)
        return fail(err, PIC_EINVAL, "unknown deposit_mode %d", p->deposit_mode);
    if (p->record_capacity < 0)
        return fail(err, PIC_EINVAL, "record_capacity must be >= 0");
    if (p->reserved != 0)
        return fail(err, PIC_EINVAL, "reserved must be 0");
    if (lds_need(p) > kMaxLds)
        return fail(err, PIC_EUNSUPPORTED, "n_cells = %d needs %zu bytes of LDS (> %zu)",
                    p->n_cells, lds_need(p), kMaxLds);
    return PIC_OK;
}

}  // namespace

struct pic_ctx {
    pic_params p;
    pic_buffers b;
    hipStream_t stream;
    Run run;
    Work wk;
    int threads;
    int poisoned;
    int64_t records_read;     // records handed out so far (step index of the next one)
    int64_t steps_done;       // steps enqueued since init
    std::string err;
    // event profiler: pairs of (class, start, stop) recorded around each launch
    int profiling;
    struct Timed { int cls; hipEvent_t a, b; };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> pool;
    double prof_ms[PIC_K_COUNT];
    int64_t prof_n[PIC_K_COUNT];
};

namespace {

// ----------------------------------------------------------- kernel dispatch tables
// kind: 0 = 1D-1V electrostatic, 1 = 1D-3V electrostatic, 2 = 1D-3V electromagnetic
int kind_of(const pic_params *p) { return is_em(p) ? 2 : (p->nv == 3 ? 1 : 0); }

template <int ORDER, int NV, bool EM>
void launch_a(pic_ctx *c, int par, int64_t step)
{
    hipLaunchKernelGGL((k_pass_a<ORDER, NV, EM>), dim3(c->run.nblocks), dim3(c->threads),
                       lds_pass_a(&c->p), c->stream, c->run, c->wk, par, step, c->b.x, c->b.v);
}

template <int ORDER, int NV, bool EM, bool PRED>
void launch_b(pic_ctx *c, int par)
{
    hipLaunchKernelGGL((k_pass_b<ORDER, NV, EM, PRED>), dim3(c->run.nblocks), dim3(c->threads),
                       lds_pass_b(&c->p), c->stream, c->run, c->wk, par, c->b.x, c->b.v, c->b.x,
                       c->b.v);
}

template <int ORDER, int NV, bool EM>
void launch_pre(pic_ctx *c)
{
    hipLaunchKernelGGL((k_predeposit<ORDER, NV, EM>), dim3(c->run.nblocks), dim3(c->threads),
                       (EM ? 3 : 1) * c->p.n_cells * 8, c->stream, c->run, c->wk, c->b.x, c->b.v);
}

enum { D_PASS_A, D_PASS_B, D_PREDEPOSIT, D_RHO };

template <int ORDER>
void dispatch_order(pic_ctx *c, int what, int par, int64_t step)
{
    const int kind = kind_of(&c->p);
    const bool pred = c->p.scheme != PIC_ESEC1;
    switch (what) {
    case D_PASS_A:
        if (kind == 0) launch_a<ORDER, 1, false>(c, par, step);
        else if (kind == 1) launch_a<ORDER, 3, false>(c, par, step);
        else launch_a<ORDER, 3, true>(c, par, step);
        break;
    case D_PASS_B:
        if (kind == 0) {
            if (pred) launch_b<ORDER, 1, false, true>(c, par);
            else launch_b<ORDER, 1, false, false>(c, par);
        } else if (kind == 1) {
            if (pred) launch_b<ORDER, 3, false, true>(c, par);
            else launch_b<ORDER, 3, false, false>(c, par);
        } else {
            launch_b<ORDER, 3, true, true>(c, par);
        }
        break;
    case D_PREDEPOSIT:
        if (kind == 0) launch_pre<ORDER, 1, false>(c);
        else if (kind == 1) launch_pre<ORDER, 3, false>(c);
        else launch_pre<ORDER, 3, true>(c);
        break;
    case D_RHO:
        hipLaunchKernelGGL((k_deposit_rho<ORDER>), dim3(c->run.nblocks), dim3(c->threads),
                           c->p.n_cells * 8, c->stream, c->run, c->wk, c->b.x);
        break;
    }
}

void dispatch(pic_ctx *c, int what, int par = 0, int64_t step = 0)
{
    if (c->p.shape_order == 1)
        dispatch_order<1>(c, what, par, step);
    else
        dispatch_order<2>(c, what, par, step);
}

int grid_threads(const pic_ctx *c)
{
    int t = 64;
    while (t < c->p.n_cells && t < 1024)
        t *= 2;
    return std::max(t, 256);
}

int check(pic_ctx *c, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->poisoned = 1;
        return fail(&c->err, PIC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    }
    return PIC_OK;
}

hipEvent_t take_event(pic_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

// Wraps one launch in a pair of events when the profiler is on.
struct Timer {
    pic_ctx *c;
    int cls;
    hipEvent_t a = nullptr;
    Timer(pic_ctx *ctx, int k) : c(ctx), cls(k)
    {
        if (c->profiling && (a = take_event(c)))
            (void)hipEventRecord(a, c->stream);
    }
    ~Timer()
    {
        if (!a)
            return;
        hipEvent_t b = take_event(c);
        if (!b) {
            c->pool.push_back(a);
            return;
        }
        (void)hipEventRecord(b, c->stream);
        c->timed.push_back({cls, a, b});
    }
};

// Accumulate the finished event pairs (the stream must be synchronised).
void collect(pic_ctx *c)
{
    for (auto &t : c->timed) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            c->prof_ms[t.cls] += ms;
            c->prof_n[t.cls] += 1;
        }
        c->pool.push_back(t.a);
        c->pool.push_back(t.b);
    }
    c->timed.clear();
}

void fill(pic_ctx *c, double *p, int64_t n, double v)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0,
                       c->stream, p, n, v);
}

}  // namespace

extern "C" {

size_t pic_workspace_size(const pic_params *p)
{
    if (validate(p, nullptr) != PIC_OK)
        return 0;
    return layout_of(p).total;
}

int pic_validate_params(const pic_params *p) { return validate(p, nullptr); }

int pic_init(const pic_params *p, const pic_buffers *b, void *hip_stream, pic_ctx **out)
{
    if (!out)
        return fail(nullptr, PIC_EINVAL, "out is NULL");
    int rc = validate(p, nullptr);
    if (rc != PIC_OK)
        return rc;
    if (!b || !b->x || !b->v || !b->E || !b->workspace)
        return fail(nullptr, PIC_EINVAL, "x, v, E and workspace must be non-NULL");
    if (is_em(p) && !b->B)
        return fail(nullptr, PIC_EINVAL, "B must be non-NULL for PIC_EMEC_LI");
    if ((p->flags & PIC_F_TRACK_IDS) && !b->id)
        return fail(nullptr, PIC_EINVAL, "PIC_F_TRACK_IDS needs an id array");
    if ((uintptr_t)b->workspace % kAlign)
        return fail(nullptr, PIC_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    const Layout L = layout_of(p);
    if (b->workspace_bytes < L.total)
        return fail(nullptr, PIC_ENOMEM, "workspace has %zu bytes, needs %zu", b->workspace_bytes, L.total);

    pic_ctx *c = new (std::nothrow) pic_ctx();
    if (!c)
        return fail(nullptr, PIC_ENOMEM, "out of host memory");
    c->p = *p;
    c->b = *b;
    c->stream = (hipStream_t)hip_stream;
    c->threads = threads_of(p);
    c->poisoned = 0;
    c->records_read = 0;
    c->steps_done = 0;
    c->profiling = 0;
    for (int k = 0; k < PIC_K_COUNT; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }

    Run &r = c->run;
    r.np = p->n_particles;
    r.ng = p->n_cells;
    r.nv = p->nv;
    r.nblocks = blocks_of(p, &r.chunk);
    r.scheme = p->scheme;
    r.pad = 0;
    r.rec_cap = records_of(p);
    r.L = p->length;
    r.h = p->length / p->n_cells;
    r.inv_h = p->n_cells / p->length;
    r.dt = p->dt;
    r.hdt = 0.5 * p->dt;
    r.c2 = p->c * p->c;
    r.qs = 1.0 / r.h;
    r.wu = p->length / (double)p->n_particles;
    for (int i = 0; i < 3; ++i)
        r.bext[i] = p->nv == 3 ? p->b_ext[i] : 0.0;
    r.w = b->w;

    char *ws = (char *)b->workspace;
    Work &w = c->wk;
    w.E = b->E;
    w.B = b->B;
    for (int k = 0; k < 2; ++k) {
        w.Ef[k] = (double *)(ws + L.Ef[k]);
        w.Bf[k] = (double *)(ws + L.Bf[k]);
        w.J1[k] = (double *)(ws + L.J1[k]);
        w.J2[k] = (double *)(ws + L.J2[k]);
    }
    w.cninv = (double *)(ws + L.cninv);
    w.spart = (double *)(ws + L.spart);
    w.st = (DevState *)(ws + L.st);
    w.rec = (DevRecord *)(ws + L.rec);

    // clear the field and current buffers (fill kernels, no memset)
    fill(c, w.Ef[0], (int64_t)(L.cninv - L.Ef[0]) / 8, 0.0);
    if (!is_em(p)) {
        // electrostatic runs carry only E_x; keep the unused components at zero
        fill(c, b->E + p->n_cells, 2 * (int64_t)p->n_cells, 0.0);
    }
    const int gt = grid_threads(c);
    if (p->nv == 1)
        hipLaunchKernelGGL((k_init_particles<1>), dim3(r.nblocks), dim3(c->threads), 0, c->stream, r, w,
                           b->x, b->v);
    else
        hipLaunchKernelGGL((k_init_particles<3>), dim3(r.nblocks), dim3(c->threads), 0, c->stream, r, w,
                           b->x, b->v);
    if (p->flags & PIC_F_INIT_GAUSS) {
        dispatch(c, D_RHO);
        hipLaunchKernelGGL(k_gauss, dim3(1), dim3(gt), 3 * p->n_cells * 8, c->stream, r, w);
    }
    if (is_em(p))
        hipLaunchKernelGGL(k_cn_init, dim3(1), dim3(gt), 0, c->stream, r, w);
    if (p->scheme != PIC_ESEC1)
        dispatch(c, D_PREDEPOSIT);
    hipLaunchKernelGGL(k_init_finish, dim3(1), dim3(gt), 0, c->stream, r, w);
    rc = check(c, "pic_init launches");
    if (rc != PIC_OK) {
        g_last_error = c->err;
        delete c;
        return rc;
    }
    *out = c;
    return PIC_OK;
}

int pic_step(pic_ctx *c, int64_t n_steps)
{
    if (!c || c->poisoned)
        return PIC_ESTATE;
    if (n_steps < 0)
        return fail(&c->err, PIC_EINVAL, "n_steps must be >= 0");
    for (int64_t s = 0; s < n_steps; ++s) {
        const int64_t n = c->steps_done;
        const int par = (int)(n & 1);
        {
            Timer t(c, PIC_K_PASS_A);
            dispatch(c, D_PASS_A, par, n);
        }
        {
            Timer t(c, PIC_K_PASS_B);
            dispatch(c, D_PASS_B, par, n);
        }
        c->steps_done = n + 1;
        if (c->profiling && c->timed.size() > 4096) {
            // bound the number of outstanding events
            if (hipStreamSynchronize(c->stream) != hipSuccess)
                return check(c, "pic_step profiler sync");
            collect(c);
        }
    }
    if (n_steps > 0)
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(grid_threads(c)), 0, c->stream, c->run, c->wk,
                           (int)(c->steps_done & 1), c->steps_done);
    return check(c, "pic_step launches");
}

int pic_diagnostics(pic_ctx *c, pic_diag *out, int64_t max_records, int64_t *n_written)
{
    if (!c || c->poisoned)
        return PIC_ESTATE;
    if (!n_written || (max_records > 0 && !out))
        return fail(&c->err, PIC_EINVAL, "out and n_written must be non-NULL");
    *n_written = 0;
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return check(c, "pic_diagnostics sync");
    DevState st;
    if (hipMemcpy(&st, c->wk.st, sizeof st, hipMemcpyDeviceToHost) != hipSuccess)
        return check(c, "pic_diagnostics state copy");
    const int64_t last = st.recorded;              // newest record
    int64_t first = c->records_read;
    if (last - first + 1 > c->run.rec_cap)
        first = last - c->run.rec_cap + 1;           // older records were overwritten
    int64_t n = std::max<int64_t>(0, std::min<int64_t>(last - first + 1, max_records));
    static_assert(sizeof(DevRecord) == sizeof(pic_diag), "record layout");
    // the records are contiguous in the ring except where it wraps: at most two copies
    int64_t done = 0;
    while (done < n) {
        const int64_t slot = (first + done) % c->run.rec_cap;
        const int64_t len = std::min<int64_t>(n - done, c->run.rec_cap - slot);
        if (hipMemcpy(out + done, c->wk.rec + slot, (size_t)len * sizeof(DevRecord),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return check(c, "pic_diagnostics record copy");
        done += len;
    }
    int nonfinite = 0;
    for (int64_t k = 0; k < n; ++k)
        nonfinite |= out[k].nonfinite;
    c->records_read = first + n;
    *n_written = n;
    return nonfinite ? PIC_ENONFINITE : PIC_OK;
}

int pic_sync_state(pic_ctx *c)
{
    if (!c || c->poisoned)
        return PIC_ESTATE;
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return check(c, "pic_sync_state");
    return PIC_OK;
}

int pic_profile_enable(pic_ctx *c, int on)
{
    if (!c || c->poisoned)
        return PIC_ESTATE;
    if (on && !c->profiling) {
        for (int k = 0; k < PIC_K_COUNT; ++k) {
            c->prof_ms[k] = 0.0;
            c->prof_n[k] = 0;
        }
    }
    c->profiling = on ? 1 : 0;
    return PIC_OK;
}

int pic_profile_read(pic_ctx *c, double *ms, int64_t *launches)
{
    if (!c || c->poisoned)
        return PIC_ESTATE;
    if (!ms || !launches)
        return fail(&c->err, PIC_EINVAL, "ms and launches must be non-NULL");
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return check(c, "pic_profile_read sync");
    collect(c);
    for (int k = 0; k < PIC_K_COUNT; ++k) {
        ms[k] = c->prof_ms[k];
        launches[k] = c->prof_n[k];
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }
    return PIC_OK;
}

int pic_destroy(pic_ctx *c)
{
    if (!c)
        return PIC_ESTATE;
    if (!c->timed.empty())
        (void)hipStreamSynchronize(c->stream);
    for (auto &t : c->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : c->pool)
        (void)hipEventDestroy(e);
    delete c;
    return PIC_OK;
}

const char *pic_strerror(int s)
{
    switch (s) {
    case PIC_OK: return "ok";
    case PIC_EINVAL: return "invalid argument";
    case PIC_ENOMEM: return "workspace too small";
    case PIC_EDEVICE: return "device error";
    case PIC_ESTATE: return "invalid context state";
    case PIC_ENONFINITE: return "non-finite value in the state";
    case PIC_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
    }
}

const char *pic_last_error(const pic_ctx *c)
{
    if (c)
        return c->err.c_str();
    return g_last_error.c_str();
}

}  // extern "C"
