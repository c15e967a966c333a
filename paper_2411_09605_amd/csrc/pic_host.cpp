// Host-only part of the PIC library runtime: parameter validation, workspace layouts,
// launch shapes and the host-side input check behind the C ABI of include/pic.h.  It uses
// no HIP: pic_lib.hip includes it into the library, and the sanitizer test builds it on
// its own with a plain C++ compiler.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/pic.h"
#include "pic_types.hpp"

using namespace pic;

namespace {

thread_local std::string g_last_error;

// Default launch: one workgroup per CU (the part has 256 CUs), 1024 threads wide.  A
// workgroup's wavefronts share its particles dynamically, which balances them only within
// the workgroup, so one workgroup per CU lets every CU finish with all of its wavefronts
// busy; more workgroups would also add prologue work and global flushes of the
// per-workgroup current tiles.  Runs with fewer than two particles per thread of such a
// launch take narrower workgroups, so that they still spread over the CUs.
constexpr int kCUs = 256;
constexpr int kDefaultThreads = 1024;
// States (x, v and the weights) larger than this interleave their batches by default: the
// Infinity Cache (256 MB) then no longer holds them between the passes, and reading one
// region of HBM at a time is faster (two-stream 4e7 particles: step -8 %); below it,
// contiguous chunks are faster.
constexpr double kInterleaveBytes = 192.0 * 1024 * 1024;
constexpr int kDefaultRecords = 4096;
// The adjoint form defaults to two 512-thread workgroups per CU once every thread gets two
// particles or more: its passes are short, and one workgroup's prologue and flush then
// overlap the other's particles (two-stream gradient, 1e6 particles, 256 cells: forward +
// backward 45.3 ms against 46.6 ms at 1024 x 256). The plain step is faster with one
// 1024-thread workgroup per CU at every size measured (1e6 to 4e7 particles).
constexpr int kAdjThreads = 512;
constexpr int kAdjGroupsPerCU = 2;
constexpr size_t kAlign = 256;
// LDS a workgroup may use on gfx950 (160 KB per CU, all of it available to one workgroup),
// less what the kernels declare statically (reduction scratch, counters: under 1 KB); this
// bounds the dynamic LDS of a launch.
constexpr size_t kMaxLds = 160 * 1024 - 1024;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool is_det(const pic_params *p) { return (p->flags & PIC_F_DETERMINISTIC) != 0; }
bool is_cc(const pic_params *p) { return (p->flags & PIC_F_CHARGE_CONSERVING) != 0; }
bool is_std(const pic_params *p) { return p->scheme == PIC_STANDARD; }

struct Layout {
    size_t Ef[2], Bf[2], J1[2], J2[2], cninv, spart, part, st, rec;
    size_t prow, ps, pf;                            // EM field launches (0 when unused)
    size_t x2, v2, id2, wcur, w2, hist, segsum;     // rebin (0 when unused)
    size_t total;
};

int threads_of(const pic_params *p)
{
    if (p->block_threads)
        return p->block_threads;
    const int64_t per_cu = (p->n_particles + kCUs - 1) / kCUs;
    int t = kDefaultThreads;
    while (t > 64 && per_cu < 2 * t)
        t /= 2;
    return t;
}

int records_of(const pic_params *p) { return p->record_capacity ? p->record_capacity : kDefaultRecords; }

int blocks_of(const pic_params *p, int64_t *chunk_out)
{
    const int t = threads_of(p);
    // default: one workgroup per CU, with at least two particles per thread
    int64_t nb = p->grid_blocks ? p->grid_blocks
                                : std::min<int64_t>(kCUs, (p->n_particles + 2 * t - 1) / (2 * t));
    nb = std::max<int64_t>(1, std::min<int64_t>(nb, kMaxGrid));
    // chunks are whole wavefronts of particles; rounding only this far keeps the number of
    // workgroups at (or one below) the one asked for, so that a grid of k workgroups per
    // compute unit loads every unit alike
    int64_t chunk = (p->n_particles + nb - 1) / nb;
    chunk = (chunk + 63) / 64 * 64;
    nb = (p->n_particles + chunk - 1) / chunk;
    if (chunk_out)
        *chunk_out = chunk;
    return (int)nb;
}

bool is_em(const pic_params *p)
{
    return p->scheme == PIC_EMEC_LI || p->scheme == PIC_EMEC_PSATD || p->scheme == PIC_EMEC_LF;
}

// EM schemes whose full-step field update is the field launch (k_em_fields)
bool has_em_fields(const pic_params *p) { return p->scheme == PIC_EMEC_LI || p->scheme == PIC_EMEC_PSATD; }

bool is_psatd(const pic_params *p) { return p->scheme == PIC_EMEC_PSATD; }

// LDS bytes of the largest kernel of this configuration.
size_t tile_width(const pic_params *p) { return (size_t)p->n_cells + 2 * kGhost; }

// LDS (bytes) of the particle passes for cells n_cells, shape order `order`; the layouts
// are those of pass_a_body and pass_b_body (tiles ghost-padded, tw = N_g + 2 kGhost).
size_t lds_pass_a_of(bool em, int order, size_t ng)
{
    const size_t tw = ng + 2 * kGhost;
    // EM: jt[3] | es[3] | bs[2] | side[3];  ES: jt | es | side | coefficients[order + 1]
    return em ? (3 + 3 + 2 + 3) * tw * 8
              : ((size_t)pic::coef_offset((int)(3 * tw)) + (order + 1) * tw) * 8;
}

size_t lds_pass_b_of(bool em, int order, size_t ng)
{
    const size_t tw = ng + 2 * kGhost;
    // EM: jt[3] | es[3] | bs[2] | eb[3] | bb[2] | e1[3] | b1[2] | CN scratch[8] | side[3]
    // ES: jt | es | eb | e1 | side | coefficients of E* and E-bar [2][order + 1]
    return em ? (3 + 3 + 2 + 3 + 2 + 3) * tw * 8 + (3 + 2 + 8) * ng * 8
              : ((size_t)pic::coef_offset((int)(4 * tw + ng)) + 2 * (order + 1) * tw) * 8;
}

// ESEC1 in one pass (esec1_body): jt | es | eb | e1[ng] | side | three coefficient tiles
size_t lds_esec1_of(int order, size_t ng)
{
    const size_t tw = ng + 2 * kGhost;
    return ((size_t)pic::coef_offset((int)(4 * tw + ng)) + 3 * (order + 1) * tw) * 8;
}

// standard scheme: the particle pass (jt | es | side | coefficient tile) and the field
// launch (rho | Green's row twice | filtered rho)
size_t lds_std_pass_of(int order, size_t ng)
{
    const size_t tw = ng + 2 * kGhost;
    return ((size_t)pic::coef_offset((int)(3 * tw)) + (order + 1) * tw) * 8;
}

size_t lds_std_field_of(size_t ng) { return 4 * ng * 8; }

// the EM field launch (k_em_fields): one pair's E, B and j, three rows and the partial
// sums of 256 threads
size_t lds_psatd_of(size_t ng) { return (6 * ng + 256) * 8; }

size_t lds_pass_a(const pic_params *p) { return lds_pass_a_of(is_em(p), p->shape_order, (size_t)p->n_cells); }

size_t lds_deposit(const pic_params *p) { return 2 * (is_em(p) ? 3 : 1) * tile_width(p) * 8; }

size_t lds_pass_b(const pic_params *p) { return lds_pass_b_of(is_em(p), p->shape_order, (size_t)p->n_cells); }

size_t lds_rebin(const pic_params *p) { return (size_t)kVBins * p->n_cells * 8; }

size_t lds_need(const pic_params *p)
{
    size_t m = p->scheme == PIC_ESEC1 ? std::max(lds_pass_a(p), lds_esec1_of(p->shape_order, (size_t)p->n_cells))
               : is_std(p) ? std::max(lds_std_pass_of(p->shape_order, (size_t)p->n_cells),
                                      lds_std_field_of((size_t)p->n_cells))
                           : std::max(lds_pass_a(p), lds_pass_b(p));
    m = std::max(m, (size_t)5 * p->n_cells * 8);   // the Gauss solve with its twiddle table
    if (has_em_fields(p))
        m = std::max(m, lds_psatd_of((size_t)p->n_cells));
    m = std::max(m, lds_deposit(p));
    if (p->rebin_every > 0)
        m = std::max(m, lds_rebin(p));
    return m;
}

// Bound on the fixed-point contributions of the LDS deposit tiles (Depo<., ., 0>): every
// tile entry receives at most one contribution per particle of a workgroup (chunk of
// them), so contributions below lim = min(2^50, 2^62 / chunk) cannot overflow 64 bits.
// The scale itself is set on the device from the particles (k_fx_setup).
void fixed_point_of(int64_t chunk, Run &r)
{
    r.fx_lim = std::min(std::ldexp(1.0, 50),
                        std::ldexp(1.0, 62) / (double)std::max<int64_t>(chunk, 1));
}

// Replicas of the current accumulators: about 32 workgroups' atomics per address (one in
// the deterministic mode, where an ordered reduction writes the current).
int nrep_of(const pic_params *p)
{
    if (is_det(p))
        return 1;
    const int nb = blocks_of(p, nullptr);
    return std::min(kMaxRep, std::max(1, (nb + 31) / 32));
}

int64_t rebin_len(const pic_params *p) { return (int64_t)kVBins * p->n_cells * blocks_of(p, nullptr); }

void scan_shape(int64_t n, int *nseg, int64_t *seg)
{
    int64_t ns = std::min<int64_t>(1024, std::max<int64_t>(1, (n + 2047) / 2048));
    *seg = (n + ns - 1) / ns;
    *nseg = (int)((n + *seg - 1) / *seg);
}

int deposit_kind(const pic_params *p)
{
    if (p->deposit_mode == PIC_DEPOSIT_LDS_ATOMIC)
        return 0;
    if (p->deposit_mode == PIC_DEPOSIT_WINDOW)
        return 1;
    if (p->deposit_mode == PIC_DEPOSIT_WAVE)
        return 2;
    if (p->deposit_mode == PIC_DEPOSIT_LDS_F64)
        return 3;
    return p->rebin_every > 0 ? 1 : 0;
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
        L.J1[k] = take((size_t)nrep_of(p) * 3 * ng * 8);
        L.J2[k] = take((size_t)nrep_of(p) * 3 * ng * 8);
    }
    L.cninv = take(ng * 8);
    L.prow = has_em_fields(p) ? take((size_t)kPsatdRows * ng * 8) : 0;
    L.ps = is_psatd(p) ? take(5 * ng * 8) : 0;
    L.pf = has_em_fields(p) ? take(5 * ng * 8) : 0;
    // two arrays of per-workgroup scalars (the one-pass ESEC1 alternates between them)
    L.spart = take(2 * (size_t)blocks_of(p, nullptr) * kNS * 8);
    L.part = is_det(p) ? take((size_t)blocks_of(p, nullptr) * 3 * ng * 8) : 0;
    L.st = take(sizeof(DevState));
    L.rec = take((size_t)records_of(p) * sizeof(DevRecord));
    L.x2 = L.v2 = L.id2 = L.wcur = L.w2 = L.hist = L.segsum = 0;
    if (p->rebin_every > 0) {
        const size_t np = (size_t)p->n_particles;
        L.x2 = take(np * 8);
        L.v2 = take(np * 8 * (size_t)p->nv);
        if (p->flags & PIC_F_TRACK_IDS)
            L.id2 = take(np * 8);
        L.wcur = take(np * 8);      // used only with non-uniform weights
        L.w2 = take(np * 8);
        L.hist = take((size_t)rebin_len(p) * 8);
        int nseg;
        int64_t seg;
        scan_shape(rebin_len(p), &nseg, &seg);
        L.segsum = take((size_t)nseg * 8);
    }
    L.total = o;
    return L;
}

int fail(std::string *where, int code, const char *fmt, ...)
    __attribute__((format(printf, 3, 4)));

constexpr int kMaxDevices = 64;   // devices whose workgroup-size check is remembered

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
    if (p->scheme < PIC_ESEC2 || p->scheme > PIC_EMEC_LF)
        return fail(err, PIC_EINVAL, "unknown scheme %d", p->scheme);
    if (p->scheme == PIC_STANDARD && !(p->flags & PIC_F_INIT_GAUSS))
        return fail(err, PIC_EINVAL, "PIC_STANDARD needs PIC_F_INIT_GAUSS (its field comes from the density)");
    if ((p->flags & PIC_F_FILTER_RHO) && p->scheme != PIC_STANDARD)
        return fail(err, PIC_EINVAL, "PIC_F_FILTER_RHO is for PIC_STANDARD only");
    if (is_em(p) && p->nv != 3)
        return fail(err, PIC_EINVAL, "the electromagnetic schemes need nv == 3");
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
    if (is_em(p) && (!(p->c > 0.0) || !std::isfinite(p->c)))
        return fail(err, PIC_EINVAL, "c must be finite and > 0 for the electromagnetic schemes");
    if (p->scheme == PIC_EMEC_LF && p->c * p->dt > p->length / p->n_cells * (1.0 + 1e-12))
        return fail(err, PIC_EINVAL, "PIC_EMEC_LF needs c dt <= h (leapfrog stability): c dt = %g, h = %g",
                    p->c * p->dt, p->length / p->n_cells);
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(p->b_ext[i]))
            return fail(err, PIC_EINVAL, "b_ext must be finite");
    if (p->rebin_every < 0)
        return fail(err, PIC_EINVAL, "rebin_every must be >= 0");
    if (p->flags & ~(uint32_t)(PIC_F_INIT_GAUSS | PIC_F_TRACK_IDS | PIC_F_INTERLEAVE |
                               PIC_F_DETERMINISTIC | PIC_F_FILTER_RHO | PIC_F_CHARGE_CONSERVING))
        return fail(err, PIC_EINVAL, "unknown flag bits 0x%x", p->flags);
    if (is_cc(p) && (p->scheme != PIC_ESEC2 || p->shape_order != 1))
        return fail(err, PIC_EINVAL, "PIC_F_CHARGE_CONSERVING needs PIC_ESEC2 and shape_order 1");
    if (is_cc(p) && (p->rebin_every > 0 || (p->deposit_mode != PIC_DEPOSIT_AUTO &&
                                            p->deposit_mode != PIC_DEPOSIT_LDS_ATOMIC &&
                                            p->deposit_mode != PIC_DEPOSIT_LDS_F64)))
        return fail(err, PIC_EINVAL,
                    "PIC_F_CHARGE_CONSERVING needs rebin_every == 0 and the LDS_ATOMIC or LDS_F64 deposit");
    if ((p->flags & PIC_F_DETERMINISTIC) && p->rebin_every > 0)
        return fail(err, PIC_EINVAL, "PIC_F_DETERMINISTIC needs rebin_every == 0");
    if ((p->flags & PIC_F_DETERMINISTIC) && p->deposit_mode != PIC_DEPOSIT_AUTO &&
        p->deposit_mode != PIC_DEPOSIT_LDS_ATOMIC)
        return fail(err, PIC_EINVAL, "PIC_F_DETERMINISTIC needs the LDS_ATOMIC deposit");
    if ((p->flags & PIC_F_INTERLEAVE) && p->rebin_every > 0)
        return fail(err, PIC_EINVAL, "PIC_F_INTERLEAVE needs rebin_every == 0");
    if (p->block_threads && (p->block_threads % 64 || p->block_threads < 64 || p->block_threads > 1024))
        return fail(err, PIC_EINVAL, "block_threads must be 0 or a multiple of 64 in [64, 1024]");
    if (p->grid_blocks < 0 || p->grid_blocks > kMaxGrid)
        return fail(err, PIC_EINVAL, "grid_blocks must be in [0, %d]", kMaxGrid);
    if (p->deposit_mode < PIC_DEPOSIT_AUTO || p->deposit_mode > PIC_DEPOSIT_LDS_F64)
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

extern "C" {

size_t pic_workspace_size(const pic_params *p)
{
    if (validate(p, nullptr) != PIC_OK)
        return 0;
    return layout_of(p).total;
}

int pic_validate_params(const pic_params *p) { return validate(p, nullptr); }

int pic_check_inputs(const pic_params *p, const double *x, const double *v, const double *w,
                     const double *E, const double *B, int64_t *bad_index)
{
    if (bad_index)
        *bad_index = -1;
    int rc = validate(p, nullptr);
    if (rc != PIC_OK)
        return rc;
    if (!x || !v || !E)
        return fail(nullptr, PIC_EINVAL, "x, v and E must be non-NULL");
    if (is_em(p) && !B)
        return fail(nullptr, PIC_EINVAL, "B must be non-NULL for the electromagnetic schemes");
    struct Array {
        const char *name;
        const double *a;
        int64_t n;
    };
    const int64_t np = p->n_particles, ng = p->n_cells;
    const Array arrays[] = {{"x", x, np},
                            {"v", v, np * p->nv},
                            {"w", w, w ? np : 0},
                            {"E", E, 3 * ng},
                            {"B", B, is_em(p) ? 2 * ng : 0}};
    for (const Array &ar : arrays)
        for (int64_t i = 0; i < ar.n; ++i)
            if (!std::isfinite(ar.a[i])) {
                if (bad_index)
                    *bad_index = i;
                return fail(nullptr, PIC_ENONFINITE, "%s[%lld] is not finite", ar.name,
                            (long long)i);
            }
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

}  // extern "C"
