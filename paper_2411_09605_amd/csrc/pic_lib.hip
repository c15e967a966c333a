// Host runtime of the PIC library: parameter validation, workspace layout, kernel
// dispatch and diagnostics behind the C ABI declared in include/pic.h.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pic.h"
#include "pic_device.hpp"
#include "pic_adjoint.hpp"

using namespace pic;

// Parameter checks, workspace layouts and launch shapes: host-only code that also builds
// on its own with a plain C++ compiler (the sanitizer test does so).
#include "pic_host.cpp"

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
    // event profiler: (class, start, stop) for each timed launch
    int profiling;
    struct Timed { int cls; hipEvent_t a, b; };
    std::vector<Timed> timed;
    hipEvent_t kev[2];        // start/stop events handed to the next particle-pass launch
    std::vector<hipEvent_t> pool;
    double prof_ms[PIC_K_COUNT];
    int64_t prof_n[PIC_K_COUNT];
};

namespace {

// LDS of the Gauss solve (gauss_body).
size_t gauss_lds(int ng) { return gauss_lds_doubles(ng) * 8; }

// ----------------------------------------------------------- kernel dispatch tables
// kind: 0 = 1D-1V electrostatic, 1 = 1D-3V electrostatic, 2 = 1D-3V electromagnetic
int kind_of(const pic_params *p) { return is_em(p) ? 2 : (p->nv == 3 ? 1 : 0); }

// Launches a particle pass; when the profiler has handed it a pair of events, the runtime
// stamps them with the start and end of this dispatch itself (no marker packets between
// kernels, so the timeline being measured is the one that runs unprofiled).
template <typename K, typename... A>
void launch_pass(pic_ctx *c, K kernel, uint32_t lds, A... args)
{
    hipEvent_t e0 = c->kev[0], e1 = c->kev[1];
    c->kev[0] = c->kev[1] = nullptr;
    hipExtLaunchKernelGGL(kernel, dim3(c->run.nblocks), dim3(c->threads), lds, c->stream, e0, e1,
                          0u, args...);
}

template <int ORDER, int NV, bool EM, int DEP>
void launch_a(pic_ctx *c, int par, int64_t step, const double *X, const double *V)
{
    launch_pass(c, k_pass_a<ORDER, NV, EM, DEP>, (uint32_t)lds_pass_a(&c->p), c->run, c->wk, par,
                step, X, V);
}

template <int ORDER, int NV, bool EM, bool PRED, int DEP>
void launch_b(pic_ctx *c, int par, const double *X, const double *V)
{
    launch_pass(c, k_pass_b<ORDER, NV, EM, PRED, DEP>, (uint32_t)lds_pass_b(&c->p), c->run, c->wk,
                par, X, V, c->b.x, c->b.v);
}

template <int ORDER, int NV, bool EM>
void launch_pre(pic_ctx *c)
{
    hipLaunchKernelGGL((k_predeposit<ORDER, NV, EM>), dim3(c->run.nblocks), dim3(c->threads),
                       lds_deposit(&c->p), c->stream, c->run, c->wk, c->b.x, c->b.v);
}

enum { D_PASS_A, D_PASS_B, D_PREDEPOSIT, D_RHO, D_ESEC1, D_STD_PASS, D_STD_PRIME };

// The three current buffers the one-pass ESEC1 rotates through (j^{n+1/2} of step n is in
// esec1_current(c, n)); ESEC1 has no predictor current, so J1[0] is the third.
double *esec1_current(pic_ctx *c, int64_t n)
{
    const int k = (int)(n % 3);
    return k == 0 ? c->wk.J2[0] : (k == 1 ? c->wk.J2[1] : c->wk.J1[0]);
}

// Which of the double-buffered fields holds the newest field after m steps: E^m in
// Ef[m & 1], or for the standard scheme E^{m-1/2} in Ef[(m - 1) & 1] (E^0 in Ef[0]).
int field_parity(const pic_ctx *c, int64_t m)
{
    if (c->p.scheme == PIC_STANDARD)
        return m > 0 ? (int)((m - 1) & 1) : 0;
    return (int)(m & 1);
}

// The per-workgroup scalars that hold the state of step m: the one-pass ESEC1 alternates
// between the two arrays; the two-pass schemes use the first.
double *spart_of(const pic_ctx *c, int64_t m)
{
    const bool alt = c->p.scheme == PIC_ESEC1 || c->p.scheme == PIC_STANDARD;
    return (alt && (m & 1)) ? c->wk.spart + (size_t)c->run.nblocks * kNS : c->wk.spart;
}

// Deterministic mode: the ordered sum of the workgroups' partial deposits into replica 0
// of J (ncomp components).
void reduce_partials(pic_ctx *c, double *J, int ncomp)
{
    const int n = ncomp * c->p.n_cells;
    hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)((n + kRedEntries - 1) / kRedEntries)),
                       dim3(256), 0, c->stream, c->wk.part, J, c->run.nblocks, n, 3 * c->p.n_cells);
}

// The standard scheme's step n: the field launch (E^{n+1/2} into Ef[n & 1] from the density
// in J2[n & 1]) and the particle pass (density of step n + 1 into J2[(n + 1) & 1]).
template <int ORDER, int NV, int DEP>
void launch_std_pass(pic_ctx *c, int64_t n, const double *X, const double *V)
{
    const int par = (int)(n & 1);
    Work wk = c->wk;
    wk.spart = spart_of(c, n);
    launch_pass(c, k_std_pass<ORDER, NV, DEP>,
                (uint32_t)lds_std_pass_of(ORDER, (size_t)c->p.n_cells), c->run, wk, par, n, X, V,
                c->b.x, c->b.v, c->wk.J2[par ^ 1], c->wk.J2[par], spart_of(c, n + 1));
}

void launch_std_field(pic_ctx *c, int64_t n)
{
    const int par = (int)(n & 1);
    hipEvent_t e0 = c->kev[0], e1 = c->kev[1];
    c->kev[0] = c->kev[1] = nullptr;
    const unsigned grid = (unsigned)((c->p.n_cells + kRedEntries - 1) / kRedEntries);
    hipExtLaunchKernelGGL(k_std_field, dim3(grid), dim3(256),
                          (uint32_t)lds_std_field_of((size_t)c->p.n_cells), c->stream, e0, e1, 0u,
                          c->run, c->wk, (const double *)c->wk.J2[par], c->wk.Ef[par],
                          (int)c->run.filter_rho);
}

// The EM field launch of step n (par = n & 1): full = 0 the predictor fields (EMEC(PSATD),
// before pass A), full = 1 the new fields and the averages pass B gathers (before pass B).
void launch_em_fields(pic_ctx *c, int par, int full)
{
    const int ng = c->p.n_cells;
    hipLaunchKernelGGL(k_em_fields, dim3((unsigned)((ng + kPsatdOut - 1) / kPsatdOut), full ? 6u : 4u),
                       dim3(kPsatdOut * kPsatdSeg), (uint32_t)lds_psatd_of((size_t)ng), c->stream,
                       c->run, c->wk, par, full);
}

template <int ORDER, int NV, int DEP>
void launch_esec1(pic_ctx *c, int64_t n, const double *X, const double *V)
{
    Work wk = c->wk;
    wk.spart = spart_of(c, n);
    launch_pass(c, k_esec1<ORDER, NV, DEP>,
                (uint32_t)lds_esec1_of(ORDER, (size_t)c->p.n_cells), c->run, wk, (int)(n & 1), n, X, V,
                c->b.x, c->b.v, (const double *)esec1_current(c, n), esec1_current(c, n + 1),
                esec1_current(c, n + 2), spart_of(c, n + 1));
}

template <int ORDER, int DEP>
void dispatch_dep(pic_ctx *c, int what, int par, int64_t step, const double *X, const double *V)
{
    const int kind = kind_of(&c->p);
    switch (what) {
    case D_ESEC1:
        if (kind == 0) launch_esec1<ORDER, 1, DEP>(c, step, X, V);
        else launch_esec1<ORDER, 3, DEP>(c, step, X, V);
        break;
    case D_STD_PASS:
        if (kind == 0) launch_std_pass<ORDER, 1, DEP>(c, step, X, V);
        else launch_std_pass<ORDER, 3, DEP>(c, step, X, V);
        break;
    case D_STD_PRIME:
        hipLaunchKernelGGL((k_std_prime<ORDER>), dim3(c->run.nblocks), dim3(c->threads),
                           lds_deposit(&c->p), c->stream, c->run, c->wk, X, V, c->wk.J2[0]);
        break;
    case D_PASS_A:
        if (kind == 0) launch_a<ORDER, 1, false, DEP>(c, par, step, X, V);
        else if (kind == 1) launch_a<ORDER, 3, false, DEP>(c, par, step, X, V);
        else launch_a<ORDER, 3, true, DEP>(c, par, step, X, V);
        break;
    case D_PASS_B:
        if (kind == 0) {
            launch_b<ORDER, 1, false, true, DEP>(c, par, X, V);
        } else if (kind == 1) {
            launch_b<ORDER, 3, false, true, DEP>(c, par, X, V);
        } else {
            launch_b<ORDER, 3, true, true, DEP>(c, par, X, V);
        }
        break;
    case D_PREDEPOSIT:
        if (kind == 0) launch_pre<ORDER, 1, false>(c);
        else if (kind == 1) launch_pre<ORDER, 3, false>(c);
        else launch_pre<ORDER, 3, true>(c);
        break;
    case D_RHO:
        hipLaunchKernelGGL((k_deposit_rho<ORDER>), dim3(c->run.nblocks), dim3(c->threads),
                           lds_deposit(&c->p), c->stream, c->run, c->wk, c->b.x);
        break;
    }
}

template <int ORDER>
void dispatch_order(pic_ctx *c, int what, int par, int64_t step, const double *X, const double *V)
{
    switch (deposit_kind(&c->p)) {
    case 3: dispatch_dep<ORDER, 3>(c, what, par, step, X, V); break;
    case 2: dispatch_dep<ORDER, 2>(c, what, par, step, X, V); break;
    case 1: dispatch_dep<ORDER, 1>(c, what, par, step, X, V); break;
    default: dispatch_dep<ORDER, 0>(c, what, par, step, X, V); break;
    }
}

void dispatch(pic_ctx *c, int what, int par = 0, int64_t step = 0, const double *X = nullptr,
              const double *V = nullptr)
{
    if (!X) {
        X = c->b.x;
        V = c->b.v;
    }
    if (c->p.shape_order == 1)
        dispatch_order<1>(c, what, par, step, X, V);
    else
        dispatch_order<2>(c, what, par, step, X, V);
    if (!c->run.det)
        return;
    const int ncur = is_em(&c->p) ? 3 : 1;
    switch (what) {
    case D_PASS_A: reduce_partials(c, c->wk.J2[par], ncur); break;
    case D_PASS_B: reduce_partials(c, c->wk.J1[par ^ 1], ncur); break;
    case D_ESEC1: reduce_partials(c, esec1_current(c, step + 1), 1); break;
    case D_STD_PASS: reduce_partials(c, c->wk.J2[(par ^ 1) & 1], 1); break;
    case D_STD_PRIME: reduce_partials(c, c->wk.J2[0], 1); break;
    case D_PREDEPOSIT: reduce_partials(c, c->wk.J1[0], ncur); break;
    case D_RHO: reduce_partials(c, c->wk.J2[0], 1); break;
    }
}

// Counting-sort rebin of the caller's state into the second buffers (x2, v2, id2, w2);
// ids and weights are copied back at once, x and v are copied back by the next pass B.
void rebin(pic_ctx *c)
{
    const int64_t n = rebin_len(&c->p);
    int nseg;
    int64_t seg;
    scan_shape(n, &nseg, &seg);
    const Run &r = c->run;
    const Work &w = c->wk;
    hipLaunchKernelGGL(k_rebin_count, dim3(r.nblocks), dim3(c->threads), lds_rebin(&c->p) / 2, c->stream,
                       r, w, c->b.x, c->b.v);
    hipLaunchKernelGGL(k_scan_sums, dim3(nseg), dim3(256), 0, c->stream, w.hist, n, seg, w.segsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, c->stream, w.segsum, nseg);
    hipLaunchKernelGGL(k_scan_apply, dim3(nseg), dim3(256), 0, c->stream, w.hist, n, seg, w.segsum);
    const int64_t *ids = (c->p.flags & PIC_F_TRACK_IDS) ? c->b.id : nullptr;
    if (c->p.nv == 1)
        hipLaunchKernelGGL((k_rebin_scatter<1>), dim3(r.nblocks), dim3(c->threads), lds_rebin(&c->p), c->stream,
                           r, w, c->b.x, c->b.v, ids);
    else
        hipLaunchKernelGGL((k_rebin_scatter<3>), dim3(r.nblocks), dim3(c->threads), lds_rebin(&c->p), c->stream,
                           r, w, c->b.x, c->b.v, ids);
    const unsigned g = (unsigned)std::min<int64_t>((r.np + 255) / 256, 4096);
    if (ids)
        hipLaunchKernelGGL(k_copy_i64, dim3(g), dim3(256), 0, c->stream, c->b.id, w.id2, r.np);
    if (w.wcur)
        hipLaunchKernelGGL(k_copy_f64, dim3(g), dim3(256), 0, c->stream, w.wcur, w.w2, r.np);
}

// Scalars and workspace arrays of one run (pic_init and the adjoint form).
void bind_run_work(const pic_params *p, const pic_buffers *b, const Layout &L, char *ws, Run &r,
                   Work &w)
{
    r.np = p->n_particles;
    r.vstride = p->n_particles;
    r.ng = p->n_cells;
    r.nv = p->nv;
    r.nblocks = blocks_of(p, &r.chunk);
    r.scheme = p->scheme;
    r.tw = (int32_t)tile_width(p);
    r.nrep = nrep_of(p);
    r.interleave = 0;
    r.det = is_det(p) ? 1 : 0;
    r.filter_rho = (p->flags & PIC_F_FILTER_RHO) ? 1 : 0;
    r.em_fields = has_em_fields(p) ? 1 : 0;
    r.cc = is_cc(p) ? 1 : 0;
    r.xshift = is_cc(p) ? 0.5 : 0.0;
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
    fixed_point_of(r.chunk, r);

    w.E = b->E;
    w.B = b->B;
    for (int k = 0; k < 2; ++k) {
        w.Ef[k] = (double *)(ws + L.Ef[k]);
        w.Bf[k] = (double *)(ws + L.Bf[k]);
        w.J1[k] = (double *)(ws + L.J1[k]);
        w.J2[k] = (double *)(ws + L.J2[k]);
    }
    w.cninv = (double *)(ws + L.cninv);
    w.prow = L.prow ? (double *)(ws + L.prow) : nullptr;
    w.ps = L.ps ? (double *)(ws + L.ps) : nullptr;
    w.pf = L.pf ? (double *)(ws + L.pf) : nullptr;
    w.grid_save = nullptr;
    w.spart = (double *)(ws + L.spart);
    w.part = L.part ? (double *)(ws + L.part) : nullptr;
    w.st = (DevState *)(ws + L.st);
    w.rec = (DevRecord *)(ws + L.rec);
    const bool rb = p->rebin_every > 0;
    w.x2 = rb ? (double *)(ws + L.x2) : nullptr;
    w.v2 = rb ? (double *)(ws + L.v2) : nullptr;
    w.id2 = (rb && (p->flags & PIC_F_TRACK_IDS)) ? (int64_t *)(ws + L.id2) : nullptr;
    w.wcur = (rb && b->w) ? (double *)(ws + L.wcur) : nullptr;
    w.w2 = (rb && b->w) ? (double *)(ws + L.w2) : nullptr;
    w.hist = rb ? (int64_t *)(ws + L.hist) : nullptr;
    w.segsum = rb ? (int64_t *)(ws + L.segsum) : nullptr;
}

int grid_threads(const pic_ctx *c)
{
    int t = 64;
    while (t < c->p.n_cells && t < 1024)
        t *= 2;
    return std::max(t, 256);
}

// The kernels read their workgroup size from the implicit kernel arguments (nthreads()).
// Check once per device that the runtime lays them out as assumed, so that a different
// layout fails here instead of giving the kernels' loops a wrong stride.
int check_group_size(hipStream_t s)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail(nullptr, PIC_EDEVICE, "hipGetDevice failed");
    static std::atomic<int> ok[kMaxDevices];
    const bool known = dev >= 0 && dev < kMaxDevices;
    if (known && ok[dev].load())
        return PIC_OK;
    hipLaunchKernelGGL(k_group_size_probe, dim3(1), dim3(64), 0, s, 0);
    hipLaunchKernelGGL(k_group_size_probe, dim3(1), dim3(256), 0, s, 1);
    int got[2] = {0, 0};
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyFromSymbolAsync(got, HIP_SYMBOL(g_group_size_probe), sizeof got, 0,
                                 hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(nullptr, PIC_EDEVICE, "workgroup-size check: %s",
                    hipGetErrorString(hipGetLastError()));
    if (got[0] != 64 || got[1] != 256)
        return fail(nullptr, PIC_EUNSUPPORTED,
                    "implicit kernel arguments not laid out as the kernels assume (group size "
                    "read as %d and %d for 64 and 256)", got[0], got[1]);
    if (known)
        ok[dev].store(1);
    return PIC_OK;
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

// Times what is enqueued in its scope when the profiler is on. A particle pass (one kernel)
// takes the two events as launch arguments and is timed from its own dispatch; a group of
// launches (the rebin) is bracketed by two recorded events.
struct Timer {
    pic_ctx *c;
    int cls;
    bool on_kernel;
    hipEvent_t a = nullptr, b = nullptr;
    Timer(pic_ctx *ctx, int k, bool one_kernel) : c(ctx), cls(k), on_kernel(one_kernel)
    {
        if (!c->profiling)
            return;
        a = take_event(c);
        b = a ? take_event(c) : nullptr;
        if (!b) {
            if (a)
                c->pool.push_back(a);
            a = nullptr;
            return;
        }
        if (on_kernel) {
            c->kev[0] = a;
            c->kev[1] = b;
        } else {
            (void)hipEventRecord(a, c->stream);
        }
    }
    ~Timer()
    {
        if (!a)
            return;
        if (on_kernel && c->kev[0] == a) {   // nothing was launched with them
            c->kev[0] = c->kev[1] = nullptr;
            c->pool.push_back(a);
            c->pool.push_back(b);
            return;
        }
        if (!on_kernel)
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

void fill_range(hipStream_t stream, double *p, int64_t n)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0,
                       stream, p, n, 0.0);
}

void fill(pic_ctx *c, double *p, int64_t n, double v)
{
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0,
                       c->stream, p, n, v);
}

// Everything pic_init does once its arguments are validated and the workspace is known to
// be large enough: bind the context to the buffers and stream and enqueue the initial
// work.  On failure the context is left for the caller to release.
int init_ctx(pic_ctx *c, const pic_params *p, const pic_buffers *b, hipStream_t stream,
             const Layout &L)
{
    if (!b->x || !b->v || !b->E)
        return fail(nullptr, PIC_EINVAL, "x, v and E must be non-NULL");
    if (is_em(p) && !b->B)
        return fail(nullptr, PIC_EINVAL, "B must be non-NULL for the electromagnetic schemes");
    if ((p->flags & PIC_F_TRACK_IDS) && !b->id)
        return fail(nullptr, PIC_EINVAL, "PIC_F_TRACK_IDS needs an id array");
    if ((uintptr_t)b->workspace % kAlign)
        return fail(nullptr, PIC_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    if (int rc = check_group_size(stream); rc != PIC_OK)
        return rc;

    c->p = *p;
    c->b = *b;
    c->stream = stream;
    c->threads = threads_of(p);
    c->poisoned = 0;
    c->records_read = 0;
    c->steps_done = 0;
    c->profiling = 0;
    c->kev[0] = c->kev[1] = nullptr;
    for (int k = 0; k < PIC_K_COUNT; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }

    bind_run_work(p, b, L, (char *)b->workspace, c->run, c->wk);
    Run &r = c->run;
    Work &w = c->wk;
    const double state_bytes = (double)p->n_particles * 8.0 * (1 + p->nv + (b->w ? 1 : 0));
    if ((p->flags & PIC_F_INTERLEAVE) || (p->rebin_every == 0 && state_bytes > kInterleaveBytes)) {
        // a workgroup then takes up to one batch more than its chunk
        constexpr int64_t umax = std::max({kUnrollA<1>, kUnrollA<3>, kUnrollB<1>, kUnrollB<3>});
        r.interleave = 1;
        fixed_point_of(r.chunk + 64 * umax, r);
    }
    if (w.wcur) {
        // the library permutes its own copy of the weights
        hipLaunchKernelGGL(k_copy_f64, dim3(1024), dim3(256), 0, c->stream, w.wcur, b->w, r.np);
        r.w = w.wcur;
    }

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
    hipLaunchKernelGGL(k_fx_setup, dim3(1), dim3(256), 0, c->stream, r, w);
    if ((p->flags & PIC_F_INIT_GAUSS) && is_cc(p)) {
        // the density with the quadratic B-spline (one degree above the tent), then Gauss'
        // law on the half-node E
        hipLaunchKernelGGL((k_deposit_rho<2>), dim3(r.nblocks), dim3(c->threads), lds_deposit(p),
                           c->stream, r, w, b->x);
        if (r.det)
            reduce_partials(c, w.J2[0], 1);
        hipLaunchKernelGGL(k_gauss_cc, dim3(1), dim3(gt), p->n_cells * 8, c->stream, r, w);
    } else if (p->flags & PIC_F_INIT_GAUSS) {
        dispatch(c, D_RHO);
        hipLaunchKernelGGL(k_gauss, dim3(1), dim3(gt), gauss_lds(p->n_cells), c->stream, r, w);
    }
    if (has_em_fields(p))
        hipLaunchKernelGGL(k_em_rows, dim3((unsigned)((p->n_cells + 255) / 256), kPsatdRows), dim3(256),
                           2 * p->n_cells * 8, c->stream, r, w);
    if (p->scheme != PIC_ESEC1)
        dispatch(c, D_PREDEPOSIT);
    hipLaunchKernelGGL(k_init_finish, dim3(1), dim3(gt), 0, c->stream, r, w);
    if (p->scheme == PIC_ESEC1)
        dispatch(c, D_PASS_A, 0, 0);    // j^{1/2}, read by the first one-pass step
    if (is_std(p)) {
        hipLaunchKernelGGL(k_std_green, dim3(1), dim3(gt), 0, c->stream, r, w);
        dispatch(c, D_STD_PRIME);       // the density at x*_0 for the first field launch
    }
    int rc = check(c, "pic_init launches");
    if (rc != PIC_OK)
        g_last_error = c->err;
    return rc;
}

// Enqueue n_steps >= 0 steps of a live context (pic_step after its argument checks).
int enqueue_steps(pic_ctx *c, int64_t n_steps)
{
    const int K = c->p.rebin_every;
    for (int64_t s = 0; s < n_steps; ++s) {
        const int64_t n = c->steps_done;
        const int par = (int)(n & 1);
        // after a rebin this step reads the sorted copy; pass B writes the caller's arrays
        const double *X = c->b.x, *V = c->b.v;
        if (K > 0 && n % K == 0) {
            Timer t(c, PIC_K_REBIN, false);
            rebin(c);
            X = c->wk.x2;
            V = c->wk.v2;
        }
        if (c->p.scheme == PIC_ESEC1) {
            Timer t(c, PIC_K_PASS_B, true);
            dispatch(c, D_ESEC1, par, n, X, V);
        } else if (is_std(&c->p)) {
            {
                Timer t(c, PIC_K_PASS_A, true);
                launch_std_field(c, n);
            }
            {
                Timer t(c, PIC_K_PASS_B, true);
                dispatch(c, D_STD_PASS, par, n, X, V);
            }
        } else {
            if (is_psatd(&c->p))
                launch_em_fields(c, par, 0);
            {
                Timer t(c, PIC_K_PASS_A, true);
                dispatch(c, D_PASS_A, par, n, X, V);
            }
            if (has_em_fields(&c->p))
                launch_em_fields(c, par, 1);
            {
                Timer t(c, PIC_K_PASS_B, true);
                dispatch(c, D_PASS_B, par, n, X, V);
            }
        }
        c->steps_done = n + 1;
        if (c->profiling && c->timed.size() > 4096) {
            // bound the number of outstanding events
            if (hipStreamSynchronize(c->stream) != hipSuccess)
                return check(c, "pic_step profiler sync");
            collect(c);
        }
    }
    if (n_steps > 0) {
        Work wk = c->wk;
        wk.spart = spart_of(c, c->steps_done);
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(grid_threads(c)), 0, c->stream, c->run, wk,
                           field_parity(c, c->steps_done), c->steps_done);
    }
    return check(c, "pic_step launches");
}

}  // namespace

extern "C" {

int pic_init(const pic_params *p, const pic_buffers *b, void *hip_stream, pic_ctx **out)
{
    if (!out)
        return fail(nullptr, PIC_EINVAL, "out is NULL");
    int rc = validate(p, nullptr);
    if (rc != PIC_OK)
        return rc;
    if (!b || !b->workspace)
        return fail(nullptr, PIC_EINVAL, "workspace must be non-NULL");
    const Layout L = layout_of(p);
    if (b->workspace_bytes < L.total)
        return fail(nullptr, PIC_ENOMEM, "workspace has %zu bytes, needs %zu", b->workspace_bytes, L.total);
    pic_ctx *c = new (std::nothrow) pic_ctx();
    if (!c)
        return fail(nullptr, PIC_ENOMEM, "out of host memory");
    rc = init_ctx(c, p, b, (hipStream_t)hip_stream, L);
    if (rc != PIC_OK) {
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
    return enqueue_steps(c, n_steps);
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

}  // extern "C"

// ----------------------------------------------------------------- checkpoint / resume
namespace {

// Layout of a saved state (host memory): this header, then the payload arrays in the
// order x[N_p], v[nv][N_p], id[N_p] (ids tracked), w[N_p] (the library's permuted copy of
// non-uniform weights, rebins only), E[3][N_g], B[2][N_g] (EM), j^{n,*} replicas
// [nrep][3][N_g].
constexpr char kStateMagic[8] = {'P', 'I', 'C', 'S', 'T', 'A', 'T', '1'};

struct StateHeader {
    char magic[8];
    int32_t abi_version, nv, scheme, shape_order;
    int64_t n_particles;
    int32_t n_cells, nrep, det, has_ids;
    int32_t has_w, pad;
    double length, dt, c, b_ext[3];
    int64_t step;          // the state is (x^n, v^n, E^n, B^n) and j^{n,*} of this step n
    DevState st;           // energies, counters and fixed-point scales
    DevRecord last;        // record of step n
    uint64_t payload_bytes;
};

struct StateParts {
    size_t x, v, id, w, E, B, J1, total;
};

StateParts state_parts(const pic_ctx *c)
{
    StateParts o;
    const size_t np = (size_t)c->p.n_particles, ng = (size_t)c->p.n_cells;
    size_t at = sizeof(StateHeader);
    auto take = [&](size_t n) { size_t a = at; at += n * 8; return a; };
    o.x = take(np);
    o.v = take(np * c->p.nv);
    o.id = (c->p.flags & PIC_F_TRACK_IDS) ? take(np) : 0;
    o.w = c->wk.wcur ? take(np) : 0;
    o.E = take(3 * ng);
    o.B = is_em(&c->p) ? take(2 * ng) : 0;
    o.J1 = take((size_t)c->run.nrep * 3 * ng);
    o.total = at;
    return o;
}

// The current a step n starts from and that only the previous step produces: j^{n,*}
// (ESEC2, EMEC(LI)) or, for the one-pass ESEC1, j^{n+1/2}.
double *carried_current(pic_ctx *c, int64_t n)
{
    if (c->p.scheme == PIC_STANDARD)
        return c->wk.J2[n & 1];     // the density at x*_n
    return c->p.scheme == PIC_ESEC1 ? esec1_current(c, n) : c->wk.J1[n & 1];
}

int copy_in(pic_ctx *c, void *dst, const void *src, size_t bytes, const char *what)
{
    if (bytes && hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, c->stream) != hipSuccess)
        return check(c, what);
    return PIC_OK;
}

}  // namespace

extern "C" {

size_t pic_state_size(const pic_ctx *c)
{
    if (!c || c->poisoned)
        return 0;
    return state_parts(c).total;
}

int pic_save_state(pic_ctx *c, void *dst, size_t bytes)
{
    if (!c || c->poisoned)
        return PIC_ESTATE;
    const StateParts sp = state_parts(c);
    if (!dst || bytes < sp.total)
        return fail(&c->err, PIC_EINVAL, "dst must hold pic_state_size() = %zu bytes", sp.total);
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return check(c, "pic_save_state sync");
    char *out = (char *)dst;
    StateHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, kStateMagic, 8);
    h.abi_version = PIC_ABI_VERSION;
    h.nv = c->p.nv;
    h.scheme = c->p.scheme;
    h.shape_order = c->p.shape_order;
    h.n_particles = c->p.n_particles;
    h.n_cells = c->p.n_cells;
    h.nrep = c->run.nrep;
    h.det = c->run.det;
    h.has_ids = (c->p.flags & PIC_F_TRACK_IDS) ? 1 : 0;
    h.has_w = c->wk.wcur ? 1 : 0;
    h.length = c->p.length;
    h.dt = c->p.dt;
    h.c = c->p.c;
    for (int i = 0; i < 3; ++i)
        h.b_ext[i] = c->p.b_ext[i];
    h.step = c->steps_done;
    h.payload_bytes = sp.total - sizeof h;
    const int par = field_parity(c, c->steps_done);
    const size_t np = (size_t)c->p.n_particles, ng = (size_t)c->p.n_cells;
    int rc = copy_in(c, &h.st, c->wk.st, sizeof h.st, "pic_save_state copy");
    if (rc == PIC_OK)
        rc = copy_in(c, &h.last, c->wk.rec + c->steps_done % c->run.rec_cap, sizeof h.last,
                     "pic_save_state copy");
    if (rc == PIC_OK) rc = copy_in(c, out + sp.x, c->b.x, np * 8, "pic_save_state copy");
    if (rc == PIC_OK) rc = copy_in(c, out + sp.v, c->b.v, np * 8 * c->p.nv, "pic_save_state copy");
    if (rc == PIC_OK && sp.id) rc = copy_in(c, out + sp.id, c->b.id, np * 8, "pic_save_state copy");
    if (rc == PIC_OK && sp.w) rc = copy_in(c, out + sp.w, c->wk.wcur, np * 8, "pic_save_state copy");
    if (rc == PIC_OK) rc = copy_in(c, out + sp.E, c->wk.Ef[par], 3 * ng * 8, "pic_save_state copy");
    if (rc == PIC_OK && sp.B) rc = copy_in(c, out + sp.B, c->wk.Bf[par], 2 * ng * 8, "pic_save_state copy");
    if (rc == PIC_OK)
        rc = copy_in(c, out + sp.J1, carried_current(c, c->steps_done),
                     (size_t)c->run.nrep * 3 * ng * 8, "pic_save_state copy");
    if (rc == PIC_OK && hipStreamSynchronize(c->stream) != hipSuccess)
        rc = check(c, "pic_save_state sync");
    if (rc != PIC_OK)
        return rc;
    std::memcpy(out, &h, sizeof h);
    return PIC_OK;
}

int pic_load_state(pic_ctx *c, const void *src, size_t bytes)
{
    if (!c || c->poisoned)
        return PIC_ESTATE;
    const StateParts sp = state_parts(c);
    if (!src || bytes < sizeof(StateHeader))
        return fail(&c->err, PIC_EINVAL, "src is NULL or shorter than a state header");
    StateHeader h;
    std::memcpy(&h, src, sizeof h);
    if (std::memcmp(h.magic, kStateMagic, 8) != 0 || h.abi_version != PIC_ABI_VERSION)
        return fail(&c->err, PIC_EINVAL, "src is not a saved state of this library version");
    bool same = h.nv == c->p.nv && h.scheme == c->p.scheme && h.shape_order == c->p.shape_order &&
                h.n_particles == c->p.n_particles && h.n_cells == c->p.n_cells &&
                h.det == c->run.det && h.has_ids == ((c->p.flags & PIC_F_TRACK_IDS) ? 1 : 0) &&
                h.has_w == (c->wk.wcur ? 1 : 0) && h.length == c->p.length && h.dt == c->p.dt &&
                h.c == c->p.c && h.step >= 0;
    for (int i = 0; i < 3; ++i)
        same = same && h.b_ext[i] == c->p.b_ext[i];
    if (!same)
        return fail(&c->err, PIC_EINVAL, "the saved state belongs to a run with other parameters");
    // the payload as this context would write it, except for the number of replicas
    const size_t ng = (size_t)c->p.n_cells, np = (size_t)c->p.n_particles;
    const size_t need = sp.total - (size_t)c->run.nrep * 3 * ng * 8 + (size_t)h.nrep * 3 * ng * 8;
    if (h.nrep < 1 || h.payload_bytes + sizeof h != need || bytes < need)
        return fail(&c->err, PIC_EINVAL, "src holds %zu bytes, the saved state needs %zu", bytes,
                    need);
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return check(c, "pic_load_state sync");
    const char *in = (const char *)src;
    const int par = field_parity(c, h.step);
    int rc = PIC_OK;
    // all current buffers start from zero; j^{n,*} is then restored
    fill(c, c->wk.J1[0], (int64_t)c->run.nrep * 3 * ng, 0.0);
    fill(c, c->wk.J1[1], (int64_t)c->run.nrep * 3 * ng, 0.0);
    fill(c, c->wk.J2[0], (int64_t)c->run.nrep * 3 * ng, 0.0);
    fill(c, c->wk.J2[1], (int64_t)c->run.nrep * 3 * ng, 0.0);
    if (rc == PIC_OK) rc = copy_in(c, c->b.x, in + sp.x, np * 8, "pic_load_state copy");
    if (rc == PIC_OK) rc = copy_in(c, c->b.v, in + sp.v, np * 8 * c->p.nv, "pic_load_state copy");
    if (rc == PIC_OK && sp.id) rc = copy_in(c, c->b.id, in + sp.id, np * 8, "pic_load_state copy");
    if (rc == PIC_OK && sp.w) rc = copy_in(c, c->wk.wcur, in + sp.w, np * 8, "pic_load_state copy");
    if (rc == PIC_OK) rc = copy_in(c, c->wk.Ef[par], in + sp.E, 3 * ng * 8, "pic_load_state copy");
    if (rc == PIC_OK) rc = copy_in(c, c->b.E, in + sp.E, 3 * ng * 8, "pic_load_state copy");
    if (rc == PIC_OK && sp.B) rc = copy_in(c, c->wk.Bf[par], in + sp.B, 2 * ng * 8, "pic_load_state copy");
    if (rc == PIC_OK && sp.B) rc = copy_in(c, c->b.B, in + sp.B, 2 * ng * 8, "pic_load_state copy");
    std::vector<double> jsum;
    if (rc == PIC_OK) {
        if (h.nrep == c->run.nrep) {
            rc = copy_in(c, carried_current(c, h.step), in + sp.J1, (size_t)h.nrep * 3 * ng * 8,
                         "pic_load_state copy");
        } else {
            // another number of replicas: their sum, in replica order, goes to replica 0
            jsum.assign(3 * ng, 0.0);
            const double *J = (const double *)(in + sp.J1);
            for (int k = 0; k < h.nrep; ++k)
                for (size_t i = 0; i < 3 * ng; ++i)
                    jsum[i] += J[(size_t)k * 3 * ng + i];
            rc = copy_in(c, carried_current(c, h.step), jsum.data(), 3 * ng * 8,
                         "pic_load_state copy");
        }
    }
    DevState st = h.st;
    st.recorded = h.step;
    st.flag_a = 0;
    if (rc == PIC_OK) rc = copy_in(c, c->wk.st, &st, sizeof st, "pic_load_state copy");
    if (rc == PIC_OK)
        rc = copy_in(c, c->wk.rec + h.step % c->run.rec_cap, &h.last, sizeof h.last,
                     "pic_load_state copy");
    if (rc == PIC_OK && hipStreamSynchronize(c->stream) != hipSuccess)
        rc = check(c, "pic_load_state sync");
    if (rc != PIC_OK)
        return rc;
    c->steps_done = h.step;
    c->records_read = h.step;
    return PIC_OK;
}

int pic_launch_shape(const pic_ctx *c, int32_t *block_threads, int32_t *grid_blocks,
                     int64_t *chunk)
{
    if (!c)
        return PIC_ESTATE;
    if (block_threads)
        *block_threads = c->threads;
    if (grid_blocks)
        *grid_blocks = c->run.nblocks;
    if (chunk)
        *chunk = c->run.chunk;
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


const char *pic_last_error(const pic_ctx *c)
{
    if (c)
        return c->err.c_str();
    return g_last_error.c_str();
}

}  // extern "C"

// =====================================================================================
// Allocation-free run
// =====================================================================================
namespace {

// Workspace of pic_run_static: one copy per device, held until the process ends.  Host
// code never passes this name to a kernel or a copy (on the host it stands for a
// host-side shadow, not the device array): it uses the device address that
// hipGetSymbolAddress returns for it, kept per device below.
static __device__ __align__(256) unsigned char scratch[PIC_STATIC_SCRATCH_BYTES];

std::atomic<void *> g_scratch_addr[kMaxDevices];

// Device address of `scratch` on the current device (looked up once per device).
int scratch_address(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail(nullptr, PIC_EDEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, PIC_EUNSUPPORTED, "device %d is beyond the %d this library tracks",
                    dev, kMaxDevices);
    void *ptr = g_scratch_addr[dev].load();
    if (!ptr) {
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(nullptr, PIC_EDEVICE, "hipGetSymbolAddress(scratch): %s",
                        hipGetErrorString(e));
        g_scratch_addr[dev].store(ptr);
    }
    *out = ptr;
    return PIC_OK;
}

}  // namespace

extern "C" {

int pic_run_static(const pic_params *p, const pic_buffers *b, void *hip_stream, int64_t n_steps,
                   pic_diag *diag_out)
{
    int rc = validate(p, nullptr);
    if (rc != PIC_OK)
        return rc;
    const Layout L = layout_of(p);
    if (L.total > (size_t)PIC_STATIC_SCRATCH_BYTES)
        return fail(nullptr, PIC_ENOMEM,
                    "this run needs %zu bytes of workspace; the static workspace holds %zu",
                    L.total, (size_t)PIC_STATIC_SCRATCH_BYTES);
    if (n_steps < 0)
        return fail(nullptr, PIC_EINVAL, "n_steps must be >= 0");
    if (!b)
        return fail(nullptr, PIC_EINVAL, "buffers are NULL");
    if (b->workspace || b->workspace_bytes)
        return fail(nullptr, PIC_EINVAL, "pic_run_static uses its own workspace: pass "
                                         "workspace = NULL and workspace_bytes = 0");
    void *ws = nullptr;
    if ((rc = scratch_address(&ws)) != PIC_OK)
        return rc;
    pic_buffers bs = *b;
    bs.workspace = ws;
    bs.workspace_bytes = PIC_STATIC_SCRATCH_BYTES;
    pic_ctx c;                      // lives for this call only
    if ((rc = init_ctx(&c, p, &bs, (hipStream_t)hip_stream, L)) != PIC_OK)
        return rc;
    if ((rc = enqueue_steps(&c, n_steps)) != PIC_OK) {
        g_last_error = c.err;
        return rc;
    }
    if (diag_out)
        hipLaunchKernelGGL(k_copy_record, dim3(1), dim3(64), 0, c.stream, c.wk, c.run.rec_cap,
                           (DevRecord *)diag_out);
    rc = check(&c, "pic_run_static launches");
    if (rc != PIC_OK)
        g_last_error = c.err;
    return rc;
}

}  // extern "C"

// =====================================================================================
// Batched ensemble form
// =====================================================================================
namespace {

constexpr int kBatchDefaultRecords = 1024;

struct BatchLayout {
    std::vector<size_t> Ef0, Ef1, Bf0, Bf1, J10, J11, J20, J21, cninv;
    size_t spart, st, rec, runs, items, stepc, total;
    int nitems;
};

int batch_threads(const pic_batch_params *p) { return p->block_threads ? p->block_threads : 256; }

int batch_chunk(const pic_batch_params *p)
{
    return p->chunk ? p->chunk : 16 * batch_threads(p);
}

int batch_records(const pic_batch_params *p)
{
    return p->record_capacity ? p->record_capacity : kBatchDefaultRecords;
}

// The per-run parameters as a single-run pic_params (for validation and LDS sizing).
pic_params run_params(const pic_batch_params *p, int r)
{
    pic_params q;
    std::memset(&q, 0, sizeof q);
    q.abi_version = PIC_ABI_VERSION;
    q.nv = p->nv;
    q.scheme = p->scheme;
    q.shape_order = p->shape_order;
    q.n_particles = p->n_particles[r];
    q.n_cells = p->n_cells[r];
    q.length = p->length[r];
    q.dt = p->dt;
    q.c = p->c;
    for (int i = 0; i < 3; ++i)
        q.b_ext[i] = p->b_ext[i];
    q.block_threads = p->block_threads;
    return q;
}

int batch_validate(const pic_batch_params *p)
{
    if (!p)
        return fail(nullptr, PIC_EINVAL, "params is NULL");
    if (p->abi_version != PIC_ABI_VERSION)
        return fail(nullptr, PIC_EINVAL, "abi_version %d != %d", p->abi_version, PIC_ABI_VERSION);
    if (p->n_runs < 1 || !p->n_particles || !p->n_cells || !p->length)
        return fail(nullptr, PIC_EINVAL, "n_runs >= 1 and the per-run arrays are required");
    if (p->flags & ~(uint32_t)PIC_BF_INIT_GAUSS)
        return fail(nullptr, PIC_EINVAL, "unknown flag bits 0x%x", p->flags);
    if (p->scheme == PIC_STANDARD || p->scheme == PIC_EMEC_PSATD || p->scheme == PIC_EMEC_LF)
        return fail(nullptr, PIC_EUNSUPPORTED, "the batched form runs ESEC2, ESEC1 and EMEC(LI)");
    if (p->block_threads && (p->block_threads % 64 || p->block_threads < 64 || p->block_threads > kBatchMaxThreads))
        return fail(nullptr, PIC_EINVAL, "block_threads must be 0 or a multiple of 64 in [64, %d]", kBatchMaxThreads);
    if (p->chunk < 0 || p->chunk % batch_threads(p))
        return fail(nullptr, PIC_EINVAL, "chunk must be 0 or a positive multiple of block_threads");
    if (p->grid_blocks < 0 || p->graph_steps < 0 || p->record_capacity < 0 || p->reserved)
        return fail(nullptr, PIC_EINVAL, "grid_blocks, graph_steps, record_capacity >= 0, reserved 0");
    int64_t items = 0;
    for (int r = 0; r < p->n_runs; ++r) {
        pic_params q = run_params(p, r);
        const int rc = validate(&q, nullptr);
        if (rc != PIC_OK)
            return fail(nullptr, rc, "run %d: %s", r, g_last_error.c_str());
        items += (q.n_particles + batch_chunk(p) - 1) / batch_chunk(p);
    }
    if (items > (int64_t)1 << 30)
        return fail(nullptr, PIC_EUNSUPPORTED, "too many work items");
    return PIC_OK;
}

// Replicas of a run's current accumulators: about 32 work items per replica.
int batch_nrep(const pic_batch_params *p, int r)
{
    const int64_t items = (p->n_particles[r] + batch_chunk(p) - 1) / batch_chunk(p);
    return (int)std::min<int64_t>(kMaxRep, std::max<int64_t>(1, (items + 31) / 32));
}

BatchLayout batch_layout(const pic_batch_params *p)
{
    BatchLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, kAlign); return at; };
    L.nitems = 0;
    for (int r = 0; r < p->n_runs; ++r) {
        const size_t ng = (size_t)p->n_cells[r];
        L.Ef0.push_back(take(3 * ng * 8));
        L.Ef1.push_back(take(3 * ng * 8));
        L.Bf0.push_back(take(2 * ng * 8));
        L.Bf1.push_back(take(2 * ng * 8));
        const size_t nr = (size_t)batch_nrep(p, r);
        L.J10.push_back(take(nr * 3 * ng * 8));
        L.J11.push_back(take(nr * 3 * ng * 8));
        L.J20.push_back(take(nr * 3 * ng * 8));
        L.J21.push_back(take(nr * 3 * ng * 8));
        L.cninv.push_back(take(ng * 8));
        L.nitems += (int)((p->n_particles[r] + batch_chunk(p) - 1) / batch_chunk(p));
    }
    L.spart = take((size_t)L.nitems * kNS * 8);
    L.st = take((size_t)p->n_runs * sizeof(DevState));
    L.rec = take((size_t)p->n_runs * batch_records(p) * sizeof(DevRecord));
    L.runs = take((size_t)p->n_runs * sizeof(BatchRun));
    L.items = take((size_t)L.nitems * sizeof(BatchItem));
    L.stepc = take(8);
    L.total = o;
    return L;
}

}  // namespace

struct pic_batch {
    pic_batch_params p;
    std::vector<int64_t> np;
    std::vector<int32_t> ng;
    std::vector<double> len;
    pic_batch_buffers b;
    hipStream_t stream;
    Batch bt;
    int threads, grid, kind;
    size_t lds_a, lds_b, lds_dep, lds_gauss;
    int64_t steps_done;
    std::vector<int64_t> records_read;
    std::vector<DevState *> st;
    std::vector<DevRecord *> rec;
    int rec_cap;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int poisoned;
    std::string err;
};

namespace {

int batch_check(pic_batch *c, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->poisoned = 1;
        return fail(&c->err, PIC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    }
    return PIC_OK;
}

template <int ORDER, int NV, bool EM>
void batch_step_kind(pic_batch *c)
{
    const bool pred = c->p.scheme != PIC_ESEC1;
    hipLaunchKernelGGL((k_batch_pass_a<ORDER, NV, EM, 0>), dim3(c->grid), dim3(c->threads), c->lds_a,
                       c->stream, c->bt);
    if (pred)
        hipLaunchKernelGGL((k_batch_pass_b<ORDER, NV, EM, true, 0>), dim3(c->grid), dim3(c->threads),
                           c->lds_b, c->stream, c->bt);
    else
        hipLaunchKernelGGL((k_batch_pass_b<ORDER, NV, EM, false, 0>), dim3(c->grid), dim3(c->threads),
                           c->lds_b, c->stream, c->bt);
    hipLaunchKernelGGL(k_batch_tick, dim3(1), dim3(64), 0, c->stream, c->bt);
}

template <int ORDER>
void batch_step_order(pic_batch *c)
{
    if (c->kind == 0) batch_step_kind<ORDER, 1, false>(c);
    else if (c->kind == 1) batch_step_kind<ORDER, 3, false>(c);
    else batch_step_kind<ORDER, 3, true>(c);
}

void batch_one_step(pic_batch *c)
{
    if (c->p.shape_order == 1)
        batch_step_order<1>(c);
    else
        batch_step_order<2>(c);
}

template <int ORDER, int NV, bool EM>
void batch_init_kind(pic_batch *c)
{
    hipLaunchKernelGGL((k_batch_init_particles<NV>), dim3(c->grid), dim3(c->threads), 0, c->stream, c->bt);
    hipLaunchKernelGGL(k_batch_fx_setup, dim3(c->p.n_runs), dim3(256), 0, c->stream, c->bt);
    if (c->p.flags & PIC_BF_INIT_GAUSS) {
        hipLaunchKernelGGL((k_batch_deposit_rho<ORDER>), dim3(c->grid), dim3(c->threads), c->lds_dep,
                           c->stream, c->bt);
        hipLaunchKernelGGL(k_batch_gauss, dim3(c->p.n_runs), dim3(512), c->lds_gauss, c->stream, c->bt);
    }
    if (EM)
        hipLaunchKernelGGL(k_batch_cn_init, dim3(c->p.n_runs), dim3(512), 0, c->stream, c->bt);
    if (c->p.scheme != PIC_ESEC1)
        hipLaunchKernelGGL((k_batch_predeposit<ORDER, NV, EM>), dim3(c->grid), dim3(c->threads),
                           c->lds_dep, c->stream, c->bt);
    hipLaunchKernelGGL(k_batch_init_finish, dim3(c->p.n_runs), dim3(512), 0, c->stream, c->bt);
}

template <int ORDER>
void batch_init_order(pic_batch *c)
{
    if (c->kind == 0) batch_init_kind<ORDER, 1, false>(c);
    else if (c->kind == 1) batch_init_kind<ORDER, 3, false>(c);
    else batch_init_kind<ORDER, 3, true>(c);
}

}  // namespace

extern "C" {

size_t pic_batch_workspace_size(const pic_batch_params *p)
{
    if (batch_validate(p) != PIC_OK)
        return 0;
    return batch_layout(p).total;
}

int pic_batch_init(const pic_batch_params *p, const pic_batch_buffers *b, void *hip_stream,
                   pic_batch **out)
{
    if (!out)
        return fail(nullptr, PIC_EINVAL, "out is NULL");
    int rc = batch_validate(p);
    if (rc != PIC_OK)
        return rc;
    const bool em = p->scheme == PIC_EMEC_LI;
    if (!b || !b->x || !b->v || !b->E || !b->workspace || (em && !b->B))
        return fail(nullptr, PIC_EINVAL, "x, v, E, workspace (and B for EM) must be non-NULL");
    if ((uintptr_t)b->workspace % kAlign)
        return fail(nullptr, PIC_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    const BatchLayout L = batch_layout(p);
    if (b->workspace_bytes < L.total)
        return fail(nullptr, PIC_ENOMEM, "workspace has %zu bytes, needs %zu", b->workspace_bytes, L.total);
    if (int rcg = check_group_size((hipStream_t)hip_stream); rcg != PIC_OK)
        return rcg;

    pic_batch *c = new (std::nothrow) pic_batch();
    if (!c)
        return fail(nullptr, PIC_ENOMEM, "out of host memory");
    c->p = *p;
    c->np.assign(p->n_particles, p->n_particles + p->n_runs);
    c->ng.assign(p->n_cells, p->n_cells + p->n_runs);
    c->len.assign(p->length, p->length + p->n_runs);
    c->p.n_particles = c->np.data();
    c->p.n_cells = c->ng.data();
    c->p.length = c->len.data();
    c->b = *b;
    c->stream = (hipStream_t)hip_stream;
    c->threads = batch_threads(p);
    c->kind = em ? 2 : (p->nv == 3 ? 1 : 0);
    c->steps_done = 0;
    c->poisoned = 0;
    c->graph = nullptr;
    c->exec = nullptr;
    c->rec_cap = batch_records(p);
    c->records_read.assign(p->n_runs, 0);

    int64_t ntot = 0;
    int maxg = 0;
    for (int r = 0; r < p->n_runs; ++r) {
        ntot += p->n_particles[r];
        maxg = std::max(maxg, p->n_cells[r]);
    }
    const int chunk = batch_chunk(p);
    char *ws = (char *)b->workspace;
    std::vector<BatchRun> runs(p->n_runs);
    std::vector<BatchItem> items;
    items.reserve(L.nitems);
    int64_t poff = 0, goff = 0;
    for (int r = 0; r < p->n_runs; ++r) {
        const pic_params q = run_params(p, r);
        BatchRun &br = runs[r];
        std::memset(&br, 0, sizeof br);
        Run &R = br.r;
        R.np = q.n_particles;
        R.vstride = ntot;
        R.ng = q.n_cells;
        R.nv = q.nv;
        R.nblocks = (int32_t)((q.n_particles + chunk - 1) / chunk);
        R.rec_cap = c->rec_cap;
        R.chunk = chunk;
        R.scheme = q.scheme;
        R.tw = q.n_cells + 2 * kGhost;
        R.nrep = batch_nrep(p, r);
        R.interleave = 0;
        R.L = q.length;
        R.h = q.length / q.n_cells;
        R.inv_h = q.n_cells / q.length;
        R.dt = q.dt;
        R.hdt = 0.5 * q.dt;
        R.c2 = q.c * q.c;
        R.qs = 1.0 / R.h;
        R.wu = q.length / (double)q.n_particles;
        fixed_point_of(chunk, R);
        for (int i = 0; i < 3; ++i)
            R.bext[i] = q.nv == 3 ? q.b_ext[i] : 0.0;
        R.w = b->w ? b->w + poff : nullptr;
        Work &W = br.wk;
        W.E = b->E + 3 * goff;
        W.B = em ? b->B + 2 * goff : nullptr;
        W.Ef[0] = (double *)(ws + L.Ef0[r]);
        W.Ef[1] = (double *)(ws + L.Ef1[r]);
        W.Bf[0] = (double *)(ws + L.Bf0[r]);
        W.Bf[1] = (double *)(ws + L.Bf1[r]);
        W.J1[0] = (double *)(ws + L.J10[r]);
        W.J1[1] = (double *)(ws + L.J11[r]);
        W.J2[0] = (double *)(ws + L.J20[r]);
        W.J2[1] = (double *)(ws + L.J21[r]);
        W.cninv = (double *)(ws + L.cninv[r]);
        W.spart = (double *)(ws + L.spart) + (size_t)items.size() * kNS;
        W.st = (DevState *)(ws + L.st) + r;
        W.rec = (DevRecord *)(ws + L.rec) + (size_t)r * c->rec_cap;
        br.poff = poff;
        c->st.push_back(W.st);
        c->rec.push_back(W.rec);
        for (int k = 0; k < R.nblocks; ++k) {
            BatchItem it;
            it.run = r;
            it.slot = k;
            it.p0 = (int64_t)k * chunk;
            it.p1 = std::min<int64_t>(q.n_particles, it.p0 + chunk);
            items.push_back(it);
        }
        poff += q.n_particles;
        goff += q.n_cells;
    }
    // largest items first: workgroups start in order as earlier ones finish, so the small
    // last items of the runs fill in at the end of each pass instead of full ones starting
    // late (the kernels find everything about an item in the item itself)
    std::stable_sort(items.begin(), items.end(), [](const BatchItem &a, const BatchItem &b) {
        return a.p1 - a.p0 > b.p1 - b.p0;
    });
    c->bt.runs = (const BatchRun *)(ws + L.runs);
    c->bt.items = (const BatchItem *)(ws + L.items);
    c->bt.nitems = (int32_t)items.size();
    c->bt.nruns = p->n_runs;
    c->bt.X = b->x;
    c->bt.V = b->v;
    c->bt.stepc = (int64_t *)(ws + L.stepc);
    c->grid = p->grid_blocks ? p->grid_blocks : std::min<int>(c->bt.nitems, 2048);

    const size_t tw = (size_t)maxg + 2 * kGhost;
    const size_t ng = (size_t)maxg;
    c->lds_a = lds_pass_a_of(em, p->shape_order, ng);
    c->lds_b = lds_pass_b_of(em, p->shape_order, ng);
    c->lds_dep = 2 * (em ? 3 : 1) * tw * 8;
    c->lds_gauss = gauss_lds((int)ng);

    if (hipMemcpy(ws + L.runs, runs.data(), runs.size() * sizeof(BatchRun), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ws + L.items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice) != hipSuccess) {
        rc = batch_check(c, "pic_batch_init table copy");
        g_last_error = c->err;
        delete c;
        return rc == PIC_OK ? PIC_EDEVICE : rc;
    }
    // clear the per-run field and current buffers
    fill_range(c->stream, (double *)(ws + L.Ef0[0]), (int64_t)(L.spart - L.Ef0[0]) / 8);
    if (!em)
        for (int r = 0; r < p->n_runs; ++r)
            fill_range(c->stream, runs[r].wk.E + p->n_cells[r], 2 * (int64_t)p->n_cells[r]);
    if (p->shape_order == 1)
        batch_init_order<1>(c);
    else
        batch_init_order<2>(c);
    rc = batch_check(c, "pic_batch_init launches");
    if (rc != PIC_OK) {
        g_last_error = c->err;
        delete c;
        return rc;
    }
    *out = c;
    return PIC_OK;
}

int pic_batch_step(pic_batch *c, int64_t n_steps)
{
    if (!c || c->poisoned)
        return PIC_ESTATE;
    if (n_steps < 0)
        return fail(&c->err, PIC_EINVAL, "n_steps must be >= 0");
    const int G = c->p.graph_steps;
    int64_t left = n_steps;
    if (G > 0 && c->stream && left >= G) {
        if (!c->exec) {
            if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return batch_check(c, "pic_batch_step capture begin");
            for (int s = 0; s < G; ++s)
                batch_one_step(c);
            if (hipStreamEndCapture(c->stream, &c->graph) != hipSuccess)
                return batch_check(c, "pic_batch_step capture end");
            if (hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0) != hipSuccess)
                return batch_check(c, "pic_batch_step graph instantiate");
        }
        while (left >= G) {
            if (hipGraphLaunch(c->exec, c->stream) != hipSuccess)
                return batch_check(c, "pic_batch_step graph launch");
            left -= G;
        }
    }
    for (; left > 0; --left)
        batch_one_step(c);
    c->steps_done += n_steps;
    if (n_steps > 0)
        hipLaunchKernelGGL(k_batch_finish, dim3(c->p.n_runs), dim3(512), 0, c->stream, c->bt);
    return batch_check(c, "pic_batch_step launches");
}

int pic_batch_diagnostics(pic_batch *c, int32_t run, pic_diag *out, int64_t max_records,
                          int64_t *n_written)
{
    if (!c || c->poisoned)
        return PIC_ESTATE;
    if (run < 0 || run >= c->p.n_runs || !n_written || (max_records > 0 && !out))
        return fail(&c->err, PIC_EINVAL, "bad run index or output pointers");
    *n_written = 0;
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return batch_check(c, "pic_batch_diagnostics sync");
    DevState st;
    if (hipMemcpy(&st, c->st[run], sizeof st, hipMemcpyDeviceToHost) != hipSuccess)
        return batch_check(c, "pic_batch_diagnostics state copy");
    const int64_t last = st.recorded;
    int64_t first = c->records_read[run];
    if (last - first + 1 > c->rec_cap)
        first = last - c->rec_cap + 1;
    const int64_t n = std::max<int64_t>(0, std::min<int64_t>(last - first + 1, max_records));
    int64_t done = 0;
    while (done < n) {
        const int64_t slot = (first + done) % c->rec_cap;
        const int64_t len = std::min<int64_t>(n - done, c->rec_cap - slot);
        if (hipMemcpy(out + done, c->rec[run] + slot, (size_t)len * sizeof(DevRecord),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return batch_check(c, "pic_batch_diagnostics record copy");
        done += len;
    }
    int nonfinite = 0;
    for (int64_t k = 0; k < n; ++k)
        nonfinite |= out[k].nonfinite;
    c->records_read[run] = first + n;
    *n_written = n;
    return nonfinite ? PIC_ENONFINITE : PIC_OK;
}

int pic_batch_destroy(pic_batch *c)
{
    if (!c)
        return PIC_ESTATE;
    if (c->exec)
        (void)hipGraphExecDestroy(c->exec);
    if (c->graph)
        (void)hipGraphDestroy(c->graph);
    delete c;
    return PIC_OK;
}

}  // extern "C"

// =====================================================================================
// Adjoint form
// =====================================================================================
namespace {

struct AdjLayout {
    Layout fwd;                      // the forward run's workspace (first)
    size_t ckx, ckv;                 // checkpoints [ncp][N_p], [ncp][N_p]
    size_t segx, segv;               // states 1..K-1 of a segment (state 0 is its
                                     // checkpoint), two segments by parity:
                                     // [2][K - 1][N_p] x2
    size_t gall;                     // every step's grids [N][6][N_g]: E^n, j^{n,*}, j^{*,n+1/2},
                                     // E*, E-bar, E^{n+1}
    size_t ax, av, lam, G1, G2, rhobar, gpart;
    size_t total;
    int ncp;
};

pic_params adj_forward_params(const pic_adj_params *p)
{
    pic_params q;
    std::memset(&q, 0, sizeof q);
    q.abi_version = PIC_ABI_VERSION;
    q.nv = 1;
    q.scheme = PIC_ESEC2;
    q.shape_order = p->shape_order;
    q.n_particles = p->n_particles;
    q.n_cells = p->n_cells;
    q.length = p->length;
    q.dt = p->dt;
    q.c = 1.0;
    q.flags = PIC_F_INIT_GAUSS;
    q.block_threads = p->block_threads;
    q.grid_blocks = p->grid_blocks;
    if (!p->block_threads && !p->grid_blocks &&
        p->n_particles >= (int64_t)2 * kAdjThreads * kAdjGroupsPerCU * kCUs) {
        q.block_threads = kAdjThreads;
        q.grid_blocks = kAdjGroupsPerCU * kCUs;
    }
    q.record_capacity = p->n_steps + 1;
    return q;
}

size_t adj_lds(const pic_params *q, int stage = 4)
{
    return adj_lds_doubles((int)tile_width(q), q->n_cells, stage) * 8;
}

int adj_validate(const pic_adj_params *p)
{
    if (!p)
        return fail(nullptr, PIC_EINVAL, "params is NULL");
    if (p->n_steps < 1 || p->checkpoint_every < 1)
        return fail(nullptr, PIC_EINVAL, "n_steps and checkpoint_every must be >= 1");
    if (p->n_modes < 0 || p->n_modes > PIC_ADJ_MAX_MODES)
        return fail(nullptr, PIC_EINVAL, "n_modes must be in [0, %d]", PIC_ADJ_MAX_MODES);
    for (int m = 0; m < p->n_modes; ++m)
        if (!std::isfinite(p->k[m]) || p->k[m] == 0.0)
            return fail(nullptr, PIC_EINVAL, "mode wavenumbers must be finite and non-zero");
    if (!std::isfinite(p->loss_weight))
        return fail(nullptr, PIC_EINVAL, "loss_weight must be finite");
    if (p->reserved[0] || p->reserved[1])
        return fail(nullptr, PIC_EINVAL, "reserved must be 0");
    const pic_params q = adj_forward_params(p);
    int rc = validate(&q, nullptr);
    if (rc != PIC_OK)
        return rc;
    if (adj_lds(&q) > kMaxLds)
        return fail(nullptr, PIC_EUNSUPPORTED, "n_cells = %d is too large for the reverse passes",
                    p->n_cells);
    return PIC_OK;
}

AdjLayout adj_layout(const pic_adj_params *p)
{
    AdjLayout A;
    const pic_params q = adj_forward_params(p);
    A.fwd = layout_of(&q);
    size_t o = A.fwd.total;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, kAlign); return at; };
    const size_t np = (size_t)p->n_particles, ng = (size_t)p->n_cells;
    const size_t K = (size_t)std::min(p->checkpoint_every, p->n_steps);
    A.ncp = (p->n_steps + p->checkpoint_every - 1) / p->checkpoint_every;
    A.ckx = take((size_t)A.ncp * np * 8);
    A.ckv = take((size_t)A.ncp * np * 8);
    A.segx = take(2 * (K - 1) * np * 8);
    A.segv = take(2 * (K - 1) * np * 8);
    A.gall = take((size_t)p->n_steps * kSaveRows * ng * 8);
    A.ax = take(np * 8);
    A.av = take(np * 8);
    A.lam = take(2 * ng * 8);
    A.G1 = take(2 * (size_t)nrep_of(&q) * ng * 8);
    A.G2 = take(2 * (size_t)nrep_of(&q) * ng * 8);
    A.rhobar = take(ng * 8);
    A.gpart = take((size_t)blocks_of(&q, nullptr) * (PIC_ADJ_MAX_MODES + 2) * 8);
    A.total = o;
    return A;
}

}  // namespace

struct pic_adj {
    pic_adj_params p;
    pic_adj_buffers b;
    pic_params q;                 // the forward run
    hipStream_t stream;
    AdjLayout A;
    Run run;
    Work wk;
    AdjWork aw;
    AdjParams ap;
    int threads;
    int forward_done;
    int poisoned;
    std::string err;
    double *ckx, *ckv, *segx, *segv, *gall;
    // the backward sweep recomputes the next segment's states on a stream of its own while
    // the caller's stream reverses the current one; events order the two
    hipStream_t side;
    hipEvent_t ev_start, ev_join, ev_rec[2], ev_rev[2];
};

namespace {

int adj_check(pic_adj *c, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->poisoned = 1;
        return fail(&c->err, PIC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    }
    return PIC_OK;
}

void adj_copy(pic_adj *c, double *dst, const double *src, int64_t n)
{
    hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0,
                       c->stream, dst, src, n);
}

template <int ORDER>
void adj_pass_a(pic_adj *c, int par, int64_t step, const double *X, const double *V)
{
    hipLaunchKernelGGL((k_pass_a<ORDER, 1, false, 0>), dim3(c->run.nblocks), dim3(c->threads),
                       lds_pass_a(&c->q), c->stream, c->run, c->wk, par, step, X, V);
}

// save: null, or where the lead workgroup copies the step's grids, E^n | j^{n,*} |
// j^{*,n+1/2} (replicas summed), and the fields built from them, E* | E-bar | E^{n+1}:
// [kSaveRows][N_g]
template <int ORDER>
void adj_pass_b(pic_adj *c, int par, const double *X, const double *V, double *Xo, double *Vo,
                double *save = nullptr)
{
    Work wk = c->wk;
    wk.grid_save = save;
    hipLaunchKernelGGL((k_pass_b<ORDER, 1, false, true, 0>), dim3(c->run.nblocks), dim3(c->threads),
                       lds_pass_b(&c->q), c->stream, c->run, wk, par, X, V, Xo, Vo);
}

// Recompute of step n of the forward run from its state (X, V) into (Xo, Vo) in one
// launch: pass B without its predictor deposit, its fields built from the grids the
// forward pass B kept (g: E^n | j^{n,*} | j^{*,n+1/2}, one replica).  The prologue forms the
// same sums in the same order as the forward run's pass B, so the new state is the
// forward run's bit for bit; pass A and both deposits are not needed again.
template <int ORDER>
void adj_recompute(pic_adj *c, hipStream_t stream, int par, const double *g, const double *X,
                   const double *V, double *Xo, double *Vo)
{
    Run r = c->run;
    r.nrep = 1;
    Work wk = c->wk;
    const int ng = c->p.n_cells;
    wk.Ef[par] = const_cast<double *>(g);
    wk.J1[par] = const_cast<double *>(g) + ng;
    wk.J2[par] = const_cast<double *>(g) + 2 * ng;
    wk.grid_save = nullptr;
    hipLaunchKernelGGL((k_pass_b<ORDER, 1, false, false, 0>), dim3(c->run.nblocks), dim3(c->threads),
                       lds_pass_b(&c->q), stream, r, wk, par, X, V, Xo, Vo);
}

template <int ORDER>
void adj_predeposit(pic_adj *c, const double *X, const double *V)
{
    hipLaunchKernelGGL((k_predeposit<ORDER, 1, false>), dim3(c->run.nblocks), dim3(c->threads),
                       lds_deposit(&c->q), c->stream, c->run, c->wk, X, V);
}

template <int ORDER, int STAGE>
void adj_rev(pic_adj *c, int q, const double *X, const double *V, const double *g,
             const double *Xm = nullptr, const double *Vm = nullptr, const double *gm = nullptr)
{
    hipLaunchKernelGGL((k_adj_reverse<ORDER, STAGE>), dim3(c->run.nblocks), dim3(c->threads),
                       adj_lds(&c->q, STAGE), c->stream, c->run, c->wk, c->aw, c->ap, q, X, V, g, Xm, Vm,
                       gm);
}

int grid_threads_of(int ng)
{
    int t = 64;
    while (t < ng && t < 1024)
        t *= 2;
    return std::max(t, 256);
}

template <int ORDER>
void adj_forward_launches(pic_adj *c)
{
    const Run &r = c->run;
    const Work &w = c->wk;
    const int ng = c->p.n_cells, gt = grid_threads_of(ng);
    double *X = c->b.x, *V = c->b.v;
    const unsigned sg = (unsigned)std::min<int64_t>((r.np + 255) / 256, 4096);
    hipLaunchKernelGGL(k_adj_sample, dim3(sg), dim3(256), 0, c->stream, r, c->ap, c->b.u, c->b.s, c->b.g,
                       X, V);
    // as pic_init: clear fields and currents, wrap, Gauss start, predictor deposit
    fill_range(c->stream, w.Ef[0], (int64_t)(c->A.fwd.cninv - c->A.fwd.Ef[0]) / 8);
    fill_range(c->stream, c->b.E + ng, 2 * (int64_t)ng);
    hipLaunchKernelGGL((k_init_particles<1>), dim3(r.nblocks), dim3(c->threads), 0, c->stream, r, w, X, V);
    hipLaunchKernelGGL(k_fx_setup, dim3(1), dim3(256), 0, c->stream, r, w);
    hipLaunchKernelGGL((k_deposit_rho<ORDER>), dim3(r.nblocks), dim3(c->threads), lds_deposit(&c->q),
                       c->stream, r, w, X);
    hipLaunchKernelGGL(k_gauss, dim3(1), dim3(gt), gauss_lds(ng), c->stream, r, w);
    adj_predeposit<ORDER>(c, X, V);
    hipLaunchKernelGGL(k_init_finish, dim3(1), dim3(gt), 0, c->stream, r, w);
    const int64_t K = c->p.checkpoint_every, N = c->p.n_steps;
    adj_copy(c, c->ckx, X, r.np);
    adj_copy(c, c->ckv, V, r.np);
    for (int64_t n = 0; n < N; ++n) {
        const int par = (int)(n & 1);
        // a checkpointed state is written by the pass B before it straight into its slot
        // and read from there; the others live in x, v
        const bool in_ck = n > 0 && n % K == 0, out_ck = (n + 1) % K == 0 && n + 1 < N;
        const double *Xi = in_ck ? c->ckx + (n / K) * r.np : X;
        const double *Vi = in_ck ? c->ckv + (n / K) * r.np : V;
        double *Xo = out_ck ? c->ckx + ((n + 1) / K) * r.np : X;
        double *Vo = out_ck ? c->ckv + ((n + 1) / K) * r.np : V;
        adj_pass_a<ORDER>(c, par, n, Xi, Vi);
        // pass B's lead keeps the step's grids and the fields built from them
        adj_pass_b<ORDER>(c, par, Xi, Vi, Xo, Vo, c->gall + n * kSaveRows * ng);
    }
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(gt), 0, c->stream, r, w, (int)(c->p.n_steps & 1),
                       (int64_t)c->p.n_steps);
    hipLaunchKernelGGL(k_adj_loss, dim3(1), dim3(256), 0, c->stream, w, r.rec_cap, (int64_t)c->p.n_steps,
                       c->p.loss_weight, c->b.loss);
}

template <int ORDER>
void adj_backward_launches(pic_adj *c)
{
    const Run &r = c->run;
    const Work &w = c->wk;
    const int ng = c->p.n_cells, N = c->p.n_steps, K = c->p.checkpoint_every;
    fill_range(c->stream, c->aw.ax, r.np);
    fill_range(c->stream, c->aw.av, r.np);
    fill_range(c->stream, c->aw.lam[0], 2 * (int64_t)ng);    // both parities
    fill_range(c->stream, c->aw.G1[0], 2 * (int64_t)r.nrep * ng);
    fill_range(c->stream, c->aw.G2[0], 2 * (int64_t)r.nrep * ng);
    // States of segment cp: its checkpoint, then the recomputed ones in the segment buffer
    // of its parity.
    const int64_t seglen = (int64_t)(std::min(K, N) - 1) * r.np;
    auto sx = [&](int cp, int j) {
        return j == 0 ? c->ckx + (int64_t)cp * r.np : c->segx + (cp & 1) * seglen + (int64_t)(j - 1) * r.np;
    };
    auto sv = [&](int cp, int j) {
        return j == 0 ? c->ckv + (int64_t)cp * r.np : c->segv + (cp & 1) * seglen + (int64_t)(j - 1) * r.np;
    };
    auto grids = [&](int cp, int j) { return c->gall + ((int64_t)cp * K + j) * kSaveRows * ng; };
    // recompute a segment's states from its checkpoint with the grids the forward run kept
    // (one gather-only launch per step), on the side stream
    auto recompute = [&](int cp) {
        const int s0 = cp * K, len = std::min(K, N - s0);
        for (int j = 0; j + 1 < len; ++j)
            adj_recompute<ORDER>(c, c->side, (int)((s0 + j) & 1), grids(cp, j), sx(cp, j), sv(cp, j),
                                 sx(cp, j + 1), sv(cp, j + 1));
        (void)hipEventRecord(c->ev_rec[cp & 1], c->side);
    };
    // the side stream starts after everything enqueued before this call
    (void)hipEventRecord(c->ev_start, c->stream);
    (void)hipStreamWaitEvent(c->side, c->ev_start, 0);
    recompute(c->A.ncp - 1);
    int q = 0;
    for (int cp = c->A.ncp - 1; cp >= 0; --cp) {
        const int s0 = cp * K, len = std::min(K, N - s0);
        if (cp > 0) {
            // the next segment's buffer was last read by the reverse of segment cp + 1
            if (cp + 1 < c->A.ncp)
                (void)hipStreamWaitEvent(c->side, c->ev_rev[(cp + 1) & 1], 0);
            recompute(cp - 1);
        }
        (void)hipStreamWaitEvent(c->stream, c->ev_rec[cp & 1], 0);
        // reverse steps of the segment: R1 of its last step, then per step R2 and R3 fused
        // with R1 of the step before (R3 alone for the segment's first step, whose
        // predecessor is in the previous segment)
        for (int j = len - 1; j >= 0; --j) {
            const double *Xj = sx(cp, j), *Vj = sv(cp, j);
            const double *g = grids(cp, j);
            if (j == len - 1)
                adj_rev<ORDER, 1>(c, q, Xj, Vj, g);
            adj_rev<ORDER, 2>(c, q, Xj, Vj, g);
            if (j > 0)
                adj_rev<ORDER, 4>(c, q, Xj, Vj, g, sx(cp, j - 1), sv(cp, j - 1), g - kSaveRows * ng);
            else
                adj_rev<ORDER, 3>(c, q, Xj, Vj, g);
            q ^= 1;
        }
        (void)hipEventRecord(c->ev_rev[cp & 1], c->stream);
    }
    // join: later work on the caller's stream follows everything on the side stream
    (void)hipEventRecord(c->ev_join, c->side);
    (void)hipStreamWaitEvent(c->stream, c->ev_join, 0);
    // reverse of the Gauss start and of the sampling
    const int gt = grid_threads_of(ng);
    hipLaunchKernelGGL(k_adj_rhobar, dim3(1), dim3(gt), gauss_lds(ng), c->stream, r, w, c->aw, q);
    hipLaunchKernelGGL((k_adj_grad<ORDER>), dim3(r.nblocks), dim3(c->threads), tile_width(&c->q) * 8,
                       c->stream, r, c->aw, c->ap, c->ckx, c->b.s, c->b.g);
    hipLaunchKernelGGL(k_adj_grad_final, dim3(1), dim3(256), 0, c->stream, c->aw, r.nblocks, c->ap.nparam,
                       c->b.grad);
}

// The side stream (default priority, on the caller's stream's device) and the events of
// the backward sweep.  Returns the first error; what was created is released by
// adj_free_side.
hipError_t adj_make_side(pic_adj *c, hipStream_t caller)
{
    c->side = nullptr;
    c->ev_start = c->ev_join = nullptr;
    c->ev_rec[0] = c->ev_rec[1] = c->ev_rev[0] = c->ev_rev[1] = nullptr;
    int dev = 0, cur = 0;
    hipError_t e = hipStreamGetDevice(caller, &dev);
    if (e == hipSuccess)
        e = hipGetDevice(&cur);
    if (e != hipSuccess)
        return e;
    if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess)
        return e;
    e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    hipEvent_t *evs[6] = {&c->ev_start, &c->ev_join, &c->ev_rec[0], &c->ev_rec[1], &c->ev_rev[0],
                          &c->ev_rev[1]};
    for (int i = 0; i < 6 && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(evs[i], hipEventDisableTiming);
    if (dev != cur) {
        const hipError_t e2 = hipSetDevice(cur);
        if (e == hipSuccess)
            e = e2;
    }
    return e;
}

void adj_free_side(pic_adj *c)
{
    if (c->side)
        (void)hipStreamSynchronize(c->side);
    hipEvent_t evs[6] = {c->ev_start, c->ev_join, c->ev_rec[0], c->ev_rec[1], c->ev_rev[0], c->ev_rev[1]};
    for (hipEvent_t ev : evs)
        if (ev)
            (void)hipEventDestroy(ev);
    if (c->side)
        (void)hipStreamDestroy(c->side);
    c->side = nullptr;
}

}  // namespace

extern "C" {

size_t pic_adj_workspace_size(const pic_adj_params *p)
{
    if (adj_validate(p) != PIC_OK)
        return 0;
    return adj_layout(p).total;
}

int pic_adj_init(const pic_adj_params *p, const pic_adj_buffers *b, void *hip_stream, pic_adj **out)
{
    if (!out)
        return fail(nullptr, PIC_EINVAL, "out is NULL");
    int rc = adj_validate(p);
    if (rc != PIC_OK)
        return rc;
    if (!b || !b->u || !b->s || !b->g || !b->x || !b->v || !b->E || !b->loss || !b->grad ||
        !b->workspace)
        return fail(nullptr, PIC_EINVAL, "every buffer must be non-NULL");
    if ((uintptr_t)b->workspace % kAlign)
        return fail(nullptr, PIC_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    const AdjLayout A = adj_layout(p);
    if (b->workspace_bytes < A.total)
        return fail(nullptr, PIC_ENOMEM, "workspace has %zu bytes, needs %zu", b->workspace_bytes, A.total);
    if (int rcg = check_group_size((hipStream_t)hip_stream); rcg != PIC_OK)
        return rcg;
    pic_adj *c = new (std::nothrow) pic_adj();
    if (!c)
        return fail(nullptr, PIC_ENOMEM, "out of host memory");
    if (adj_make_side(c, (hipStream_t)hip_stream) != hipSuccess) {
        adj_free_side(c);
        delete c;
        (void)hipGetLastError();
        return fail(nullptr, PIC_EDEVICE, "could not create the adjoint's side stream and events");
    }
    c->p = *p;
    c->b = *b;
    c->q = adj_forward_params(p);
    c->stream = (hipStream_t)hip_stream;
    c->A = A;
    c->threads = threads_of(&c->q);
    c->forward_done = 0;
    c->poisoned = 0;
    char *ws = (char *)b->workspace;
    pic_buffers fb;
    std::memset(&fb, 0, sizeof fb);
    fb.x = b->x;
    fb.v = b->v;
    fb.E = b->E;
    fb.workspace = b->workspace;
    fb.workspace_bytes = A.fwd.total;
    bind_run_work(&c->q, &fb, A.fwd, ws, c->run, c->wk);
    c->ckx = (double *)(ws + A.ckx);
    c->ckv = (double *)(ws + A.ckv);
    c->segx = (double *)(ws + A.segx);
    c->segv = (double *)(ws + A.segv);
    c->gall = (double *)(ws + A.gall);
    AdjWork &aw = c->aw;
    const int ng = p->n_cells;
    aw.ax = (double *)(ws + A.ax);
    aw.av = (double *)(ws + A.av);
    for (int k = 0; k < 2; ++k) {
        aw.lam[k] = (double *)(ws + A.lam) + k * ng;
        aw.G1[k] = (double *)(ws + A.G1) + (size_t)k * c->run.nrep * ng;
        aw.G2[k] = (double *)(ws + A.G2) + (size_t)k * c->run.nrep * ng;
    }
    aw.rhobar = (double *)(ws + A.rhobar);
    aw.gpart = (double *)(ws + A.gpart);
    std::memset(&c->ap, 0, sizeof c->ap);
    c->ap.n_modes = p->n_modes;
    c->ap.nparam = p->n_modes + 2;
    for (int m = 0; m < p->n_modes; ++m)
        c->ap.k[m] = p->k[m];
    *out = c;
    return PIC_OK;
}

int pic_adj_forward(pic_adj *c, const double *alpha, double v_beam, double v_spread)
{
    if (!c || c->poisoned)
        return PIC_ESTATE;
    if ((c->p.n_modes > 0 && !alpha) || !std::isfinite(v_beam) || !std::isfinite(v_spread))
        return fail(&c->err, PIC_EINVAL, "alpha must be given and the speeds finite");
    double asum = 0.0;
    for (int m = 0; m < c->p.n_modes; ++m) {
        if (!std::isfinite(alpha[m]))
            return fail(&c->err, PIC_EINVAL, "alpha must be finite");
        asum += std::fabs(alpha[m]);
        c->ap.alpha[m] = alpha[m];
    }
    if (asum >= 1.0)
        return fail(&c->err, PIC_EINVAL, "sum |alpha_m| must be < 1 (positive density)");
    c->ap.v_beam = v_beam;
    c->ap.v_spread = v_spread;
    if (c->p.shape_order == 1)
        adj_forward_launches<1>(c);
    else
        adj_forward_launches<2>(c);
    c->forward_done = 1;
    return adj_check(c, "pic_adj_forward launches");
}

int pic_adj_backward(pic_adj *c, double loss_bar)
{
    if (!c || c->poisoned)
        return PIC_ESTATE;
    if (!c->forward_done)
        return fail(&c->err, PIC_ESTATE, "pic_adj_backward needs a forward run first");
    if (!std::isfinite(loss_bar))
        return fail(&c->err, PIC_EINVAL, "loss_bar must be finite");
    c->ap.lbw = loss_bar * c->p.loss_weight * c->run.h;
    if (c->p.shape_order == 1)
        adj_backward_launches<1>(c);
    else
        adj_backward_launches<2>(c);
    return adj_check(c, "pic_adj_backward launches");
}

int pic_adj_records(pic_adj *c, pic_diag *out, int64_t max_records, int64_t *n_written)
{
    if (!c || c->poisoned)
        return PIC_ESTATE;
    if (!n_written || (max_records > 0 && !out))
        return fail(&c->err, PIC_EINVAL, "out and n_written must be non-NULL");
    *n_written = 0;
    if (hipStreamSynchronize(c->stream) != hipSuccess)
        return adj_check(c, "pic_adj_records sync");
    if (!c->forward_done)
        return PIC_OK;
    const int64_t n = std::min<int64_t>(c->p.n_steps + 1, max_records);
    if (n > 0 && hipMemcpy(out, c->wk.rec, (size_t)n * sizeof(DevRecord), hipMemcpyDeviceToHost) != hipSuccess)
        return adj_check(c, "pic_adj_records copy");
    *n_written = n;
    return PIC_OK;
}

int pic_adj_destroy(pic_adj *c)
{
    if (!c)
        return PIC_ESTATE;
    adj_free_side(c);
    delete c;
    return PIC_OK;
}

}  // extern "C"
