// Device code of the explicit energy-conserving PIC step for gfx950 (CDNA4).
//
// Particle state is a structure of FP64 arrays (x[N_p], v[nv][N_p]) streamed from HBM
// with one lane per particle; the 1D grid (a few hundred nodes) lives in LDS for the
// whole pass.  One step of ESEC2 / EMEC(LI) (eq. (good_translation), (EMbasic)) is two
// kernel launches:
//
//   pass A: every workgroup builds the predictor fields E* (B*) in LDS from E^n (B^n)
//           and the predictor current j^{n,*}; per particle x* = x + dt/2 v, gather at
//           x*, v*, x^{n+1}, x^{n+1/2} = (x^n + x^{n+1}) / 2, deposit w v* at x^{n+1/2}
//           into an LDS tile; the tile is added to the global current with FP64 atomics
//   pass B: every workgroup rebuilds E* (bit-identically) and builds E^{n+1} (B^{n+1})
//           and the averaged fields from the centred current (Ampere / Crank-Nicolson);
//           per particle it recomputes x*, v*, x^{n+1/2}, gathers the averaged fields at
//           x^{n+1/2}, forms v-dagger and Gamma (eq. (opt_solution)) with the fallback,
//           writes x^{n+1} (wrapped) and v^{n+1}, and - because x*_{n+1} = x^{n+1} +
//           dt/2 v^{n+1} is then known - deposits the NEXT step's predictor current
//           w v^{n+1} at x*_{n+1}; the last workgroup stores E^{n+1} (B^{n+1}) and W_E, W_B
//
// The grid work is tiny (N_g nodes) and is repeated by every workgroup in its prologue,
// which costs a few microseconds of L2 reads and saves the single-workgroup kernels and
// the grid-wide synchronisation they would need.  Fields and currents are double
// buffered by step parity.  The particle state is read twice and written once per step
// (48 B per particle in 1D-1V, 96 B in 1D-3V).  Recomputing v* in pass B instead of
// storing it keeps the deposit in pass A and the gather in pass B at exactly the same
// x^{n+1/2} (the code is compiled without FP contraction), which is what the energy
// identity of eq. (exp_econs_simple) needs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pic_types.hpp"

namespace pic {

// Particles whose loads each thread issues together before computing on them, per pass
// (more loads in flight against fewer waves per SIMD from the extra registers).
template <int NV> constexpr int kUnrollA = 2;
template <int NV> constexpr int kUnrollB = 2;
// Minimum wavefronts per SIMD the particle passes are compiled for: 6 for 1D-1V (at most 80
// VGPRs, so memory, LDS and ALU work of more wavefronts overlap); 1D-3V keeps its registers.
template <int NV> constexpr int kWavesPerEU = NV == 1 ? 6 : 1;
// Largest workgroup of the particle passes.
template <int NV> constexpr int kMaxThreads = 1024;

// Run::scheme of the electromagnetic schemes, EMEC(LI), EMEC(PSATD) and EMEC(LF).
__host__ __device__ constexpr bool em_scheme(int s) { return s == 2 || s == kPsatd || s == kLeapfrog; }

// Threads of the (1-D) workgroup: the group-size field of the implicit kernel arguments
// (a 16-bit field at byte 12), read with a scalar load of the dword that holds it.
// blockDim.x also allows for a partial last workgroup, which these launches never have,
// and is read with a vector load; vector loads complete in order, so waiting for it
// would also wait for every particle load issued before it.  (The dispatch packet holds
// the same number but may sit in host memory.)
__device__ __forceinline__ unsigned nthreads()
{
    typedef const __attribute__((address_space(4))) unsigned int *kernarg_ptr;
    return ((kernarg_ptr)__builtin_amdgcn_implicitarg_ptr())[3] & 0xffffu;
}

// Written by k_group_size_probe: nthreads() as read in one-workgroup launches of 64 and
// 256 threads (the library checks them once per device before its first launch).
__device__ int g_group_size_probe[2];

__global__ void k_group_size_probe(int slot)
{
    if (threadIdx.x == 0)
        g_group_size_probe[slot] = (int)nthreads();
}

// A thread's batch of U particles (lane l of a wavefront takes b + l + 64 u, u < U; see
// BatchAddr), loaded together.  The particle loops keep the next batch's loads in flight
// while they compute on the current one (and the first batch's loads in flight during the
// field prologue), so HBM latency overlaps LDS and ALU work.
template <int U, int NV> struct PBatch {
    double x[U], v[U][NV];
};

// Addressing of a wavefront's batch of 64 U consecutive particles starting at `start` (the
// same in every lane): lane l takes start + l + 64 u.  Entries past p1 are clamped to
// particle p1 - 1 (every range holds at least one particle), so loads are issued without a
// per-lane branch.  The base is wavefront-uniform and the per-lane offset 32-bit, which
// lets the loads use a scalar base register instead of 64-bit vector address arithmetic.
struct BatchAddr {
    int64_t b0;        // first particle of the batch, clamped to p1 - 1
    unsigned lim;      // largest offset inside [b0, p1)
    __device__ __forceinline__ BatchAddr(int64_t start, int64_t p1, unsigned span)
    {
        b0 = min(start, p1 - 1);
        lim = (unsigned)min(p1 - 1 - b0, (int64_t)(span - 1));
    }
    __device__ __forceinline__ unsigned off(unsigned lane, int u) const
    {
        return min(lane + 64u * (unsigned)u, lim);
    }
};

// Loads the batch at `start` (U particles per lane).  The compiler then knows how many
// loads are in flight and lets the next batch load while the current one is processed.
// Callers mask the entries past p1 with their own bounds test.
template <int U, int NV>
__device__ __forceinline__ void load_batch(PBatch<U, NV> &b, const double *__restrict__ X,
                                           const double *__restrict__ V, int64_t vstride,
                                           int64_t start, int64_t p1)
{
    const BatchAddr a(start, p1, 64u * U);
    const unsigned lane = threadIdx.x & 63;
    const double *Xb = X + a.b0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const unsigned o = a.off(lane, u);
        b.x[u] = Xb[o];
#pragma unroll
        for (int c = 0; c < NV; ++c)
            b.v[u][c] = (V + c * vstride + a.b0)[o];
    }
}

// Weights of the batch at `start` (W[p], or wu when W is null).  Issued before the next
// batch's loads, so that waiting for them does not wait for the prefetch.
template <int U>
__device__ __forceinline__ void load_weights(double (&w)[U], const double *__restrict__ W,
                                             double wu, int64_t start, int64_t p1)
{
    const BatchAddr a(start, p1, 64u * U);
    const unsigned lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < U; ++u)
        w[u] = W ? (W + a.b0)[a.off(lane, u)] : wu;
}

// A workgroup's particles go to its wavefronts in batches of 64 U consecutive particles
// (lane l takes b + l + 64 u): wavefront w starts with the workgroup's batch w, and each
// then claims the next unclaimed batch from a counter in LDS.  The hardware issues older
// wavefronts first, so a fixed split leaves the youngest ones finishing alone at the end
// of the pass; claiming batches as they go, the wavefronts of a workgroup finish within
// about one batch of each other.  The counter is set by reset() before a barrier that
// precedes the first claim.
//
// Batch k of a workgroup starts at origin + k step.  Chunks (the default): the
// workgroup's particles are [p0, p1), origin = p0 and step = one batch.  Interleaved:
// batches are dealt to the workgroups round-robin, origin = b batches for workgroup b
// and step = nblocks batches, so that at any moment the grid reads one region of the
// state rather than nblocks separate ones; with the state streaming from HBM this reads
// faster, with it in the Infinity Cache the chunks do (callers pass p1 = N_p).
//
// Static (the deterministic mode): wavefront w takes batches w, w + W, w + 2W, ... of
// its workgroup's W wavefronts, so every thread always sees the same particles in the
// same order and its running sums (kinetic energy) are reproducible bit for bit.
template <int U> struct WaveBatches {
    static constexpr int kBatch = 64 * U;
    int64_t origin, step;
    int64_t np, last;      // reversed order: batch start s maps to last - s while s < np
    int *ctr;
    int fixed;             // 1: static assignment
    int k;                 // static: index of the wavefront's current batch
    // Interleaved runs (the state larger than the 256 MB Infinity Cache) can walk the state
    // from its end (reverse): a pass that starts where the previous pass ended finds up to
    // 256 MB of the state still in the cache.  The set of batches is the same either way.
    __device__ __forceinline__ WaveBatches(int64_t p0, int *counter, int interleave = 0,
                                           int nblocks = 1, int static_order = 0,
                                           int64_t n_particles = 0, bool reverse = false)
        : ctr(counter), fixed(static_order)
    {
        origin = interleave ? (int64_t)blockIdx.x * kBatch : p0;
        step = interleave ? (int64_t)nblocks * kBatch : (int64_t)kBatch;
        k = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        np = (interleave && reverse && n_particles > 0) ? n_particles : 0;
        last = np > 0 ? (np - 1) / kBatch * kBatch : 0;
    }
    __device__ __forceinline__ int64_t order(int64_t s) const
    {
        return s < np ? last - s : s;
    }
    __device__ __forceinline__ void reset() const
    {
        if (threadIdx.x == 0)
            *ctr = (int)(nthreads() >> 6);
    }
    // first particle of this wavefront's first batch (the same in every lane)
    __device__ __forceinline__ int64_t first() const
    {
        return order(origin + (int64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * step);
    }
    // claim the next batch (every lane of the wavefront active)
    __device__ __forceinline__ int64_t claim()
    {
        if (fixed) {
            k += (int)(nthreads() >> 6);
            return order(origin + (int64_t)k * step);
        }
        int kc = 0;
        if ((threadIdx.x & 63) == 0)
            kc = atomicAdd(ctr, 1);
        return order(origin + (int64_t)__builtin_amdgcn_readlane(kc, 0) * step);
    }
};

// ------------------------------------------------------------------ shape functions
// Cardinal B-spline weights of degree ORDER for a particle at xi = x / h - shift
// (section 2.2).  first = index of the leftmost node of the ORDER + 1 node stencil.
template <int ORDER> struct Stencil {
    int first;
    double w[ORDER + 1];
};

__device__ __forceinline__ Stencil<1> stencil1(double xi)
{
    double f = floor(xi);
    double d = xi - f;
    Stencil<1> s;
    s.first = (int)f;
    s.w[0] = 1.0 - d;
    s.w[1] = d;
    return s;
}

// Quadratic weights (1/2 - d)^2 / 2, 3/4 - d^2, (1/2 + d)^2 / 2, expanded as
// t -+ d/2 with t = 1/8 + d^2/2 (five operations; gather and deposit share them).
__device__ __forceinline__ Stencil<2> stencil2(double xi)
{
    double f = floor(xi + 0.5);
    double d = xi - f;                       // in [-1/2, 1/2)
    double hd = 0.5 * d;
    double t = fma(hd, d, 0.125);
    Stencil<2> s;
    s.first = (int)f - 1;
    s.w[0] = t - hd;
    s.w[1] = fma(-d, d, 0.75);
    s.w[2] = t + hd;
    return s;
}

template <int ORDER> __device__ __forceinline__ Stencil<ORDER> stencil(double xi);
template <> __device__ __forceinline__ Stencil<1> stencil<1>(double xi) { return stencil1(xi); }
template <> __device__ __forceinline__ Stencil<2> stencil<2>(double xi) { return stencil2(xi); }

// Periodic node index.  Positions handed to the passes are within a few cells of
// [0, L), so the first two tests decide; the modulo keeps any input (even NaN, which
// converts to an arbitrary int) inside the tile.
__device__ __forceinline__ int wrap_node(int i, int ng)
{
    if ((unsigned)i < (unsigned)ng)
        return i;
    if (i < 0 && i >= -ng)
        return i + ng;
    if (i >= ng && i < 2 * ng)
        return i - ng;
    int r = i % ng;
    return r < 0 ? r + ng : r;
}

// LDS tiles hold N_g nodes plus kGhost periodic copies on each side: node i of
// component c sits at slot c * tw + kGhost + i (tw = N_g + 2 kGhost).  The ORDER + 1
// slots of a stencil are always consecutive: a stencil whose nodes fall inside the padded
// range indexes the tile directly, and one beyond the ghost band has its first node
// wrapped into [0, N_g), which keeps the rest inside the right ghost band (ORDER <=
// kGhost).  So the LDS accesses of one stencil share a base address.
static_assert(kGhost >= 2, "a wrapped quadratic stencil must fit the right ghost band");
template <int ORDER> struct Slots {
    int n[ORDER + 1];
};

template <int ORDER>
__device__ __forceinline__ Slots<ORDER> slots_of(const Stencil<ORDER> &s, int ng)
{
    int b = s.first + kGhost;
    if ((unsigned)b > (unsigned)(ng + 2 * kGhost - ORDER - 1))
        b = wrap_node(s.first, ng) + kGhost;
    Slots<ORDER> o;
#pragma unroll
    for (int k = 0; k <= ORDER; ++k)
        o.n[k] = b + k;
    return o;
}

__device__ __forceinline__ int slot_of_node(int i, int ng)
{
    return (unsigned)(i + kGhost) < (unsigned)(ng + 2 * kGhost) ? i + kGhost
                                                                 : wrap_node(i, ng) + kGhost;
}

template <int ORDER>
__device__ __forceinline__ double gather1(const double *tile, const Stencil<ORDER> &s,
                                          const Slots<ORDER> &n)
{
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k <= ORDER; ++k)
        acc = fma(tile[n.n[k]], s.w[k], acc);
    return acc;
}

// Gathers that deposit nothing at the same position use the field as a polynomial in the
// particle's offset d inside its cell (d as in stencil<ORDER>): sum_k E_k w_k(d) expanded
// once per cell in the prologue, so a gather costs ORDER FMAs instead of the weights and
// ORDER + 1 FMAs.  Coefficient tile: slot s holds the ORDER + 1 coefficients of the cell
// whose stencil starts at slot s.
template <int ORDER> struct Cell {
    int base;            // slot of the stencil's first node
    double d;
};

template <int ORDER> __device__ __forceinline__ Cell<ORDER> cell_of(double xi, int ng)
{
    const double f = floor(ORDER == 2 ? xi + 0.5 : xi);
    Cell<ORDER> c;
    c.d = xi - f;
    Stencil<ORDER> s;
    s.first = (int)f - (ORDER == 2 ? 1 : 0);
    c.base = slots_of<ORDER>(s, ng).n[0];
    return c;
}

template <int ORDER>
__device__ __forceinline__ double gather_poly(const double *ct, const Cell<ORDER> &c)
{
    const double *k = ct + (ORDER + 1) * c.base;
    if constexpr (ORDER == 1)
        return fma(c.d, k[1], k[0]);
    else
        return fma(c.d, fma(c.d, k[2], k[1]), k[0]);
}

// Coefficients of every cell of a tile from its interior t[0..ng) (periodic).
//   tent:      E(d) = E_0 + d (E_1 - E_0)
//   quadratic: E(d) = (E_0 + E_2)/8 + 3 E_1/4 + d (E_2 - E_0)/2 + d^2 ((E_0 + E_2)/2 - E_1)
template <int ORDER>
__device__ __forceinline__ void coef_fill(double *ct, const double *t, int ng, int tw)
{
    for (int s = threadIdx.x; s < tw - ORDER; s += nthreads()) {
        const double e0 = t[wrap_node(s - kGhost, ng)], e1 = t[wrap_node(s - kGhost + 1, ng)];
        if constexpr (ORDER == 1) {
            ct[2 * s] = e0;
            ct[2 * s + 1] = e1 - e0;
        } else {
            const double e2 = t[wrap_node(s - kGhost + 2, ng)];
            ct[3 * s] = 0.125 * (e0 + e2) + 0.75 * e1;
            ct[3 * s + 1] = 0.5 * (e2 - e0);
            ct[3 * s + 2] = 0.5 * (e0 + e2) - e1;
        }
    }
}


// Add a workgroup's ghost-padded LDS current tile (ncomp components) into the global
// current (hardware FP64 atomics); ghost slots go to their periodic nodes, zero entries
// (common when the particles are cell-sorted) are skipped.
__device__ __forceinline__ void tile_flush(const double *tile, double *J, int ncomp, int ng,
                                           int tw)
{
    for (int idx = threadIdx.x; idx < ncomp * tw; idx += nthreads()) {
        const double val = tile[idx];
        if (val != 0.0) {
            const int c = idx / tw, j = idx % tw;
            unsafeAtomicAdd(&J[c * ng + wrap_node(j - kGhost, ng)], val);
        }
    }
}

// Deposit accumulator of one thread for NC current components (tile stride tw).
// DEP = 0: each particle adds its ORDER + 1 contributions with LDS atomics on a 64-bit
//          fixed-point tile (below).
// DEP = 1 (particles cell-sorted, so a thread's successive particles share a cell or
//          two): contributions are summed in registers over a window of ORDER + 3 nodes
//          anchored one node left of the stencil that opened it, and added to the tile
//          only when a particle's stencil leaves the window, and at the end.
// DEP = 2: a register window shared by the wavefront (below).
// DEP = 3: each particle adds its contributions with FP64 LDS atomics.
// Every kind has init(side, run), add(...), finish(tile, tw, ng); after the workgroup has
// synchronised, flush_tile(tile, J, ncomp, ng, tw) adds the tile into the global current.
template <int ORDER, int NC, int DEP> struct Depo;

// DEP = 0.  A contribution c is stored as round(c 2^S): one FMA against 1.5 2^52 rounds
// c 2^S to an integer exactly while |c 2^S| < 2^51, and the integer is added with
// ds_add_u64, which runs at about twice the rate of FP64 LDS atomics on random addresses.
// Sums inside a workgroup are then exact and independent of the order of the adds.  The
// scale 2^S is chosen at initialisation (k_fx_setup) so that twice the largest
// contribution of the initial particles, 2 max_p w_p |v_p| / h, stays below Run::fx_lim
// (<= 2^62 / chunk): each entry receives at most one contribution per particle of the
// workgroup, so no entry can overflow.  A contribution at or beyond the bound (a particle
// more than twice as fast as the fastest initial one, or a non-finite value) leaves the
// fixed-point path:
//   default            - it is added to an FP64 side tile with FP64 LDS atomics;
//   deterministic mode - it is rounded to a coarser fixed point, 2^(S - kFxCoarse), in the
//                        same side tile (as integers; exact and order-independent too),
//                        while |c| 2^(S - kFxCoarse) < fx_lim; beyond that (or not finite)
//                        it is dropped and `over` is set (the step is then reported as
//                        non-finite).
constexpr double kFxMagic = 6755399441055744.0;   // 1.5 * 2^52
constexpr int kFxCoarse = 12;

__device__ __forceinline__ long long fx_round(double v)
{
    return __double_as_longlong(v + kFxMagic) - __double_as_longlong(kFxMagic);
}

template <int ORDER, int NC> struct Depo<ORDER, NC, 0> {
    double *side;
    double scale, lim, inv;
    int det;
    int over;              // deterministic mode: a contribution was out of range
    __device__ __forceinline__ void init(double *side_tile, const Run &r, const DevState *st,
                                         int which = 0)
    {
        side = side_tile;
        scale = st->fx_scale[which];
        inv = st->fx_inv[which];
        lim = r.fx_lim;
        det = r.det;
        over = 0;
    }
    __device__ __forceinline__ void add(double *jt, int tw, int ng, const Stencil<ORDER> &s,
                                        const double (&q)[NC], bool = true, bool = true)
    {
        const Slots<ORDER> sl = slots_of<ORDER>(s, ng);
        unsigned long long *ti = reinterpret_cast<unsigned long long *>(jt);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double qs = q[c] * scale;
            if (fabs(qs) < lim) {
#pragma unroll
                for (int k = 0; k <= ORDER; ++k) {
                    const double m = fma(qs, s.w[k], kFxMagic);
                    const long long iv = __double_as_longlong(m) - __double_as_longlong(kFxMagic);
                    atomicAdd(&ti[c * tw + sl.n[k]], (unsigned long long)iv);
                }
            } else if (!det) {
#pragma unroll
                for (int k = 0; k <= ORDER; ++k)
                    atomicAdd(&side[c * tw + sl.n[k]], q[c] * s.w[k]);
            } else {
                const double qc = qs * (1.0 / (double)(1 << kFxCoarse));
                if (fabs(qc) < lim) {
                    unsigned long long *si = reinterpret_cast<unsigned long long *>(side);
#pragma unroll
                    for (int k = 0; k <= ORDER; ++k)
                        atomicAdd(&si[c * tw + sl.n[k]], (unsigned long long)fx_round(qc * s.w[k]));
                } else {
                    over = 1;
                }
            }
        }
    }
    __device__ __forceinline__ void finish(double *, int, int) {}
    // Tile slot `idx` as a double: the integer sum times 2^-S plus the side tile.
    __device__ __forceinline__ double value(const double *jt, int idx) const
    {
        const double fine = (double)__double_as_longlong(jt[idx]) * inv;
        if (!det)
            return fine + side[idx];
        return fine + (double)__double_as_longlong(side[idx]) * (inv * (double)(1 << kFxCoarse));
    }
    // Default: each entry back to a double on its way into the global current (FP64
    // atomics).  Deterministic mode: J is this workgroup's row of the partial sums; node i
    // receives its interior slot and its periodic ghost images, added in slot order.
    __device__ __forceinline__ void flush_tile(const double *jt, double *J, int ncomp, int ng,
                                               int tw)
    {
        if (det) {
            for (int idx = threadIdx.x; idx < ncomp * ng; idx += nthreads()) {
                const int c = idx / ng, i = idx % ng;
                double acc = 0.0;
                for (int j = (i + kGhost) % ng; j < tw; j += ng)
                    acc += value(jt, c * tw + j);
                J[c * ng + i] = acc;
            }
            return;
        }
        for (int idx = threadIdx.x; idx < ncomp * tw; idx += nthreads()) {
            const double val = value(jt, idx);
            if (val != 0.0) {
                const int c = idx / tw, j = idx % tw;
                unsafeAtomicAdd(&J[c * ng + wrap_node(j - kGhost, ng)], val);
            }
        }
    }
};

template <int ORDER, int NC> struct Depo<ORDER, NC, 3> {
    int over = 0;
    __device__ __forceinline__ void init(double *, const Run &, const DevState *, int = 0) {}
    __device__ __forceinline__ void add(double *jt, int tw, int ng, const Stencil<ORDER> &s,
                                        const double (&q)[NC], bool = true, bool = true)
    {
        const Slots<ORDER> sl = slots_of<ORDER>(s, ng);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int k = 0; k <= ORDER; ++k)
                atomicAdd(&jt[c * tw + sl.n[k]], q[c] * s.w[k]);
    }
    __device__ __forceinline__ void finish(double *, int, int) {}
    __device__ __forceinline__ void flush_tile(const double *jt, double *J, int ncomp, int ng,
                                               int tw)
    {
        tile_flush(jt, J, ncomp, ng, tw);
    }
};


template <int ORDER, int NC> struct Depo<ORDER, NC, 1> {
    static constexpr int W = ORDER + 3;
    int anchor;
    bool live;
    int over = 0;
    double acc[NC][W];
    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int j = 0; j < W; ++j)
                acc[c][j] = 0.0;
    }
    __device__ __forceinline__ void init(double *, const Run &, const DevState *, int = 0)
    {
        live = false;
        anchor = 0;
        clear();
    }
    __device__ __forceinline__ void flush_tile(const double *jt, double *J, int ncomp, int ng,
                                               int tw)
    {
        tile_flush(jt, J, ncomp, ng, tw);
    }
    __device__ __forceinline__ void flush(double *jt, int tw, int ng)
    {
        if (!live)
            return;
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const int slot = slot_of_node(anchor + j, ng);
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (acc[c][j] != 0.0)
                    atomicAdd(&jt[c * tw + slot], acc[c][j]);
        }
        clear();
    }
    __device__ __forceinline__ void add(double *jt, int tw, int ng, const Stencil<ORDER> &s,
                                        const double (&q)[NC], bool = true, bool = true)
    {
        int d = s.first - anchor;
        if (!live || d < 0 || d > W - ORDER - 1) {
            flush(jt, tw, ng);
            anchor = s.first - 1;
            live = true;
            d = 1;
        }
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double a = 0.0;
#pragma unroll
            for (int k = 0; k <= ORDER; ++k)
                if (j - k >= 0 && j - k <= W - ORDER - 1)
                    a = (d == j - k) ? s.w[k] : a;
#pragma unroll
            for (int c = 0; c < NC; ++c)
                acc[c][j] = fma(q[c], a, acc[c][j]);
        }
    }
    __device__ __forceinline__ void finish(double *jt, int tw, int ng) { flush(jt, tw, ng); }
};

// Cross-lane move within rows of 16 lanes (DPP), for a double.
template <int CTRL> __device__ __forceinline__ double dpp_mov(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront (all lanes active): butterflies within rows of 16
// with DPP (quad permutations, half-row and row mirrors), then across rows.
__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_mov<0xB1>(v);     // quad_perm [1, 0, 3, 2]
    v += dpp_mov<0x4E>(v);     // quad_perm [2, 3, 0, 1]
    v += dpp_mov<0x141>(v);    // row_half_mirror
    v += dpp_mov<0x140>(v);    // row_mirror
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// DEP = 2 (particles cell-sorted; every lane of the wavefront calls add, with `valid`
// false past the end of the range): each lane sums its contributions in registers over a
// window of ORDER + 3 nodes shared by the whole wavefront.  The window is placed one node
// left of the stencil of the wavefront's first particle and stays put while that stencil
// remains inside it (sub-cell wobble does not move it); when it leaves, the window is
// summed across the wavefront (DPP) and one lane adds it to the LDS tile.  A run of
// sorted particles thus costs a few LDS atomics per wavefront instead of ORDER + 1 per
// particle.  A lane whose stencil is outside the window adds it with LDS atomics.  The
// window may move only at calls with `may_move` (the first particle of each batch), so
// the reduction code appears once in the unrolled particle loop.
template <int ORDER, int NC> struct Depo<ORDER, NC, 2> {
    static constexpr int W = ORDER + 3;
    int anchor;            // the same in every lane of the wavefront
    bool live;
    int over = 0;
    double acc[NC][W];
    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int j = 0; j < W; ++j)
                acc[c][j] = 0.0;
    }
    __device__ __forceinline__ void init(double *, const Run &, const DevState *, int = 0)
    {
        live = false;
        anchor = 0;
        clear();
    }
    __device__ __forceinline__ void flush_tile(const double *jt, double *J, int ncomp, int ng,
                                               int tw)
    {
        tile_flush(jt, J, ncomp, ng, tw);
    }
    // all lanes of the wavefront active
    __device__ __forceinline__ void flush(double *jt, int tw, int ng)
    {
        if (!live)
            return;
        const bool lead = (threadIdx.x & 63) == 0;
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const int slot = slot_of_node(anchor + j, ng);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double t = wave_sum_dpp(acc[c][j]);
                if (lead && t != 0.0)
                    atomicAdd(&jt[c * tw + slot], t);
            }
        }
        clear();
    }
    __device__ __forceinline__ void add(double *jt, int tw, int ng, const Stencil<ORDER> &s,
                                        const double (&q)[NC], bool valid, bool may_move)
    {
        if (may_move) {
            // lane 0 holds the wavefront's lowest particle index; invalid lanes are the
            // highest ones, so an invalid lane 0 means the whole wavefront is past the end
            const int f0 = __builtin_amdgcn_readfirstlane(s.first);
            const int v0 = __builtin_amdgcn_readfirstlane((int)valid);
            const int d0 = f0 - anchor;
            if (v0 && (!live || d0 < 0 || d0 > W - ORDER - 1)) {
                flush(jt, tw, ng);
                anchor = f0 - 1;
                live = true;
            }
        }
        if (!valid)
            return;
        if (!live) {
            // (only before the first window is placed) add directly
            const Slots<ORDER> sl = slots_of<ORDER>(s, ng);
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int k = 0; k <= ORDER; ++k)
                    atomicAdd(&jt[c * tw + sl.n[k]], q[c] * s.w[k]);
            return;
        }
        const int d = s.first - anchor;
        if (d >= 0 && d <= W - ORDER - 1) {
#pragma unroll
            for (int j = 0; j < W; ++j) {
                double a = 0.0;
#pragma unroll
                for (int k = 0; k <= ORDER; ++k)
                    if (j - k >= 0 && j - k <= W - ORDER - 1)
                        a = (d == j - k) ? s.w[k] : a;
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    acc[c][j] = fma(q[c], a, acc[c][j]);
            }
        } else {
            const Slots<ORDER> sl = slots_of<ORDER>(s, ng);
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int k = 0; k <= ORDER; ++k)
                    atomicAdd(&jt[c * tw + sl.n[k]], q[c] * s.w[k]);
        }
    }
    __device__ __forceinline__ void finish(double *jt, int tw, int ng) { flush(jt, tw, ng); }
};

// Periodic position in [0, L).  A particle moves less than a period per step, so one
// conditional add or subtract almost always suffices; otherwise x - L floor(x / L),
// with rounding that lands on L mapped to 0.
__device__ __forceinline__ double wrap_pos(double x, double L)
{
    if (x < 0.0)
        x += L;
    else if (x >= L)
        x -= L;
    if (x < 0.0 || x >= L || !(x == x)) {
        x = x - L * floor(x / L);
        if (x < 0.0)
            x += L;
        if (x >= L)
            x = 0.0;
    }
    return x;
}

// Exact charge conservation (section 3.5; Run::cc; tent shapes): the centred current and
// v-dagger's field go through the pieces of the particle's path x0 -> x1 (x0 wrapped, as
// stored; x1 unwrapped) between the half nodes, where the tent has its kinks.  In
// u = x / h - 1/2 the half nodes are the integers; a piece [s, e] is visited at its
// midpoint with the fraction (e - s) / |u1 - u0| of the path (on a piece the tent is
// linear, so its value at the midpoint is its time average there, and eq. (detbal) holds
// piece by piece).  Coordinates are taken relative to the whole cell `base` = floor(u0),
// and the end point as its wrapped image's u plus the whole periods in between: that is
// the number the next step starts from, whereas x / h itself is not exactly periodic in
// floating point (over many boundary crossings the difference would drift Gauss' law).
// visit(base, t, frac) gets the midpoint t relative to base.  A path with no length, or
// one longer than 2^30 cells (only a non-finite or absurd state), is one piece.
template <typename F>
__device__ __forceinline__ void cc_pieces(const Run &r, double x0, double x1, F &&visit)
{
    const double ua = x0 * r.inv_h - 0.5;
    const double base = floor(ua);
    const double xw = wrap_pos(x1, r.L);
    // whole periods between x1 and xw (x1 - xw is a multiple of L up to rounding, so the
    // reciprocal of L, inv_h / N_g, serves)
    const double m = rint((x1 - xw) * (r.inv_h / (double)r.ng));
    const double ta = ua - base;
    const double tb = (xw * r.inv_h - 0.5) + (m * (double)r.ng - base);
    const double lo = fmin(ta, tb), hi = fmax(ta, tb), len = hi - lo;
    if (!(len > 0.0) || !(len < 1073741824.0)) {
        visit(base, 0.5 * (ta + tb), 1.0);
        return;
    }
    const double il = 1.0 / len;                    // one division per path
    double t = lo;
    for (;;) {
        const double e = fmin(floor(t) + 1.0, hi);
        visit(base, 0.5 * (t + e), (e - t) * il);
        if (e >= hi)
            break;
        t = e;
    }
}

// Tent stencil at u = base + t (base a whole number).
__device__ __forceinline__ Stencil<1> cc_stencil(double base, double t)
{
    const double f = floor(t);
    const double d = t - f;
    Stencil<1> s;
    s.first = (int)(base + f);
    s.w[0] = 1.0 - d;
    s.w[1] = d;
    return s;
}

// v-dagger's field through the pieces of the path x0 -> x1 (tent coefficient tile ct).
__device__ __forceinline__ double cc_gather(const Run &r, const double *ct, double x0, double x1)
{
    double acc = 0.0;
    cc_pieces(r, x0, x1, [&](double base, double t, double f) {
        const Stencil<1> st = cc_stencil(base, t);
        Cell<1> c;
        c.base = slots_of<1>(st, r.ng).n[0];
        c.d = st.w[1];
        acc = fma(f, gather_poly<1>(ct, c), acc);
    });
    return acc;
}


// --------------------------------------------------------------- block reductions
// Workgroup barrier that orders LDS only.  __syncthreads also waits for every global load
// and store the wavefront has in flight (particle writes, the last prefetch), which costs
// microseconds at the end of a pass; exchanges through LDS need only the LDS operations
// complete.  Global memory written before it is not made visible to the workgroup.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum (max) over the 64 lanes of a wavefront, all lanes active; every lane gets the same
// value.  Within each row of 16 lanes, DPP butterflies (quad permutations, half-row and row
// mirrors) leave the row's sum in all of its lanes (each addition pairs the same two
// values in both lanes, so the lanes agree bit for bit); the four row sums are then read
// from lanes 0, 16, 32, 48 and combined in that order.  No LDS round trips.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_mov<0xB1>(v);     // quad_perm [1, 0, 3, 2]
    v += dpp_mov<0x4E>(v);     // quad_perm [2, 3, 0, 1]
    v += dpp_mov<0x141>(v);    // row_half_mirror
    v += dpp_mov<0x140>(v);    // row_mirror
    return ((read_lane(v, 0) + read_lane(v, 16)) + read_lane(v, 32)) + read_lane(v, 48);
}

__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp_mov<0xB1>(v));
    v = fmax(v, dpp_mov<0x4E>(v));
    v = fmax(v, dpp_mov<0x141>(v));
    v = fmax(v, dpp_mov<0x140>(v));
    return fmax(fmax(fmax(read_lane(v, 0), read_lane(v, 16)), read_lane(v, 32)), read_lane(v, 48));
}

// LDS for the block reductions: up to 4 values per wavefront of a 1024-thread workgroup.
constexpr int kRedSize = 64;
// Ordered sums over many rows (k_reduce_partials, k_std_field): a workgroup of 256 threads
// takes kRedEntries consecutive entries, kRedSegments threads per entry.
constexpr int kRedEntries = 32, kRedSegments = 8;

// Deterministic reduction of N values over the workgroup in one round of LDS: value k is
// summed, or maximised where bit k of MAXMASK is set, always in the same fixed order for a
// given blockDim (so a value gives the same result whatever is reduced beside it); every
// thread gets the results.  red: kRedSize doubles of LDS.  The barriers order LDS only.
template <unsigned MAXMASK, int N>
__device__ __forceinline__ void block_reduce(double (&v)[N], double *red)
{
    static_assert(N >= 1 && N * 16 <= kRedSize, "reduction too wide");
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (nthreads() + 63) >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k)
        v[k] = (MAXMASK >> k) & 1u ? wave_max(v[k]) : wave_sum(v[k]);
    lds_barrier();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k)
            red[k * 16 + wid] = v[k];
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double *rk = red + k * 16;
        double t;
        if ((MAXMASK >> k) & 1u) {
            t = rk[0];
            for (int i = 1; i < nw; ++i)
                t = fmax(t, rk[i]);
        } else {
            t = 0.0;
            for (int i = 0; i < nw; ++i)
                t += rk[i];
        }
        v[k] = t;
    }
    lds_barrier();
}

__device__ __forceinline__ double block_sum(double v, double *red)
{
    double a[1] = {v};
    block_reduce<0u>(a, red);
    return a[0];
}

__device__ __forceinline__ double block_max(double v, double *red)
{
    double a[1] = {v};
    block_reduce<1u>(a, red);
    return a[0];
}

// Mean of n values (LDS or global), identical in every workgroup of a launch.
__device__ __forceinline__ double block_mean(const double *a, int n, double *red)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += nthreads())
        s += a[i];
    return block_sum(s, red) / n;
}


// Component value J[i] summed over nrep <= kMaxRep replicas of stride rs, in replica
// order; the loads are issued together.
__device__ __forceinline__ double rep_sum(const double *J, int i, int nrep, int rs)
{
    double a[kMaxRep];
#pragma unroll
    for (int k = 0; k < kMaxRep; ++k)
        a[k] = k < nrep ? J[(size_t)k * rs + i] : 0.0;
    double s = a[0];
#pragma unroll
    for (int k = 1; k < kMaxRep; ++k)
        s += a[k];
    return s;
}

// Sum of the replicas of the first n values of J into dst (LDS or global).
__device__ __forceinline__ void rep_gather(double *dst, const double *J, int n, int nrep, int rs)
{
    for (int i = threadIdx.x; i < n; i += nthreads())
        dst[i] = rep_sum(J, i, nrep, rs);
}

// Zero every replica of the first n values of J.
__device__ __forceinline__ void rep_zero(double *J, int n, int nrep, int rs)
{
    for (int k = 0; k < nrep; ++k)
        for (int i = threadIdx.x; i < n; i += nthreads())
            J[(size_t)k * rs + i] = 0.0;
}

// Zero part `part` of `nparts` of every replica of the first n values of J (the parts
// together cover them once), so that all workgroups of a launch share the clearing.
__device__ __forceinline__ void rep_zero_part(double *J, int n, int nrep, int rs, int64_t part,
                                              int64_t nparts)
{
    const int64_t tot = (int64_t)nrep * n;
    const int64_t per = (tot + nparts - 1) / nparts;
    const int64_t e1 = min(tot, (part + 1) * per);
    for (int64_t e = part * per + threadIdx.x; e < e1; e += nthreads())
        J[(e / n) * rs + e % n] = 0.0;
}

// The replica a workgroup adds into.
__device__ __forceinline__ double *rep_slot(double *J, int nrep, int ng)
{
    return J + (size_t)(blockIdx.x % nrep) * 3 * ng;
}

// Where a workgroup's deposit tile goes: its replica of the current J, or in the
// deterministic mode its own row of the partial sums (k_reduce_partials then writes J).
__device__ __forceinline__ double *dep_target(const Run &r, const Work &wk, double *J)
{
    return r.det ? wk.part + (size_t)blockIdx.x * 3 * r.ng : rep_slot(J, r.nrep, r.ng);
}

// A deterministic-mode deposit met a value it cannot hold: report it with the next record.
template <typename D> __device__ __forceinline__ void flag_over(const D &dep, const Work &wk)
{
    if (dep.over)
        atomicOr(&wk.st->flag_a, 1);
}

__device__ __forceinline__ void tile_load(double *dst, const double *src, int n)
{
    for (int i = threadIdx.x; i < n; i += nthreads())
        dst[i] = src[i];
}

__device__ __forceinline__ void tile_zero(double *dst, int n)
{
    for (int i = threadIdx.x; i < n; i += nthreads())
        dst[i] = 0.0;
}

// Fill the ghost slots of ncomp tile components from their periodic images (the
// interior must be written and visible).
__device__ __forceinline__ void ghost_fill(double *tile, int ncomp, int ng, int tw)
{
    for (int idx = threadIdx.x; idx < ncomp * 2 * kGhost; idx += nthreads()) {
        const int c = idx / (2 * kGhost), j = idx % (2 * kGhost);
        const int slot = j < kGhost ? j : ng + j;
        tile[c * tw + slot] = tile[c * tw + wrap_node(slot - kGhost, ng) + kGhost];
    }
}

// Interiors of the ghost-padded E [3][tw] and B [2][tw] tiles from a field block
// E [3][ng] | B [2][ng] (Work::ps or Work::pf); the caller fills the ghosts.
__device__ __forceinline__ void psatd_tiles(const Run &r, const double *src, double *et, double *bt)
{
    const int ng = r.ng, tw = r.tw;
    for (int idx = threadIdx.x; idx < 5 * ng; idx += nthreads()) {
        const int c = idx / ng, i = idx - c * ng;
        double *dst = c < 3 ? et + c * tw : bt + (c - 3) * tw;
        dst[kGhost + i] = src[idx];
    }
}

// ------------------------------------------------------------------ grid operations
// Staggered differences: nodes f[i] at i h, half nodes g[i] at (i + 1/2) h.
__device__ __forceinline__ double dplus(const double *f, int i, int ng, double inv_h)
{
    return (f[i + 1 == ng ? 0 : i + 1] - f[i]) * inv_h;
}
__device__ __forceinline__ double dminus(const double *g, int i, int ng, double inv_h)
{
    return (g[i] - g[i == 0 ? ng - 1 : i - 1]) * inv_h;
}

// EMEC(LF) magnetic half step at half node i, component c (0: B_y, 1: B_z):
// B^{n+1/2} = B^{n-1/2} - dt curl E^n, (curl E)_y = -D+E_z, (curl E)_z = D+E_y
// (eq. (EMleapfrog), second line).  E [3][ng], B [2][ng] in global memory.
__device__ __forceinline__ double lf_bhalf(const Run &r, const double *E, const double *B, int c,
                                           int i)
{
    const int ng = r.ng, ip = i + 1 == ng ? 0 : i + 1;
    if (c == 0)
        return B[i] + r.dt * ((E[2 * ng + ip] - E[2 * ng + i]) * r.inv_h);
    return B[ng + i] - r.dt * ((E[ng + ip] - E[ng + i]) * r.inv_h);
}

// EMEC(LF)'s magnetic energy of the state (E^n, B^{n-1/2}) (section 4.1):
// W_B^n = c^2/2 h sum B^{n+1/2} . B^{n-1/2}.  Summed by the first wavefront in an order
// fixed by N_g alone (the other wavefronts add exact zeros), so that every writer of a
// record (a pass's lead, the end-of-call launch, initialisation) gets the same bits.
// Every thread gets the result.
__device__ __forceinline__ double lf_magnetic_energy(const Run &r, const double *E, const double *B,
                                                     double *red)
{
    const int ng = r.ng;
    double s = 0.0;
    if (threadIdx.x < 64)
        for (int idx = threadIdx.x; idx < 2 * ng; idx += 64) {
            const int c = idx >= ng ? 1 : 0, i = idx - c * ng;
            s = fma(lf_bhalf(r, E, B, c, i), B[idx], s);
        }
    return 0.5 * r.c2 * r.h * block_sum(s, red);
}

// Predictor fields into the interiors of the LDS tiles es [ne][tw], bs [2][tw] from E^n,
// B^n and j^{n,*} (the caller fills the ghosts):
//   ESEC2: E* = E - dt/2 (j - mean j)                        (eq. (good_translation))
//   EM   : E* = E + dt/2 (c^2 curl B - j), B* = B - dt/2 curl E   (eq. (EMbasic))
//   EMEC(LF): B^{n+1/2} = B - dt curl E into bs, E* = E + dt/2 (c^2 curl B^{n+1/2} - j)
//          (eq. (EMleapfrog); the workgroup synchronises between the two)
//   ESEC1: E* = E  (v* uses E^n, eq. (naivetranslation))
// In 1D: (curl B)_y = -D-B_z, (curl B)_z = D-B_y, (curl E)_y = -D+E_z, (curl E)_z = D+E_y.
__device__ __forceinline__ void predictor_fields(const Run &r, const double *E, const double *B,
                                 const double *J, double *es, double *bs, double *red, int nrep)
{
    const int ng = r.ng, tw = r.tw, rs = 3 * ng;
    double *e0 = es + kGhost, *b0 = bs + kGhost;
    if (r.scheme == 1) {
        for (int i = threadIdx.x; i < ng; i += nthreads())
            e0[i] = E[i];
        return;
    }
    if (r.scheme == 0) {
        // the summed current goes through the tile (each thread rereads its own entries)
        for (int i = threadIdx.x; i < ng; i += nthreads())
            e0[i] = rep_sum(J, i, nrep, rs);
        const double mean = block_mean(e0, ng, red);
        for (int i = threadIdx.x; i < ng; i += nthreads())
            e0[i] = E[i] - r.hdt * (e0[i] - mean);
        return;
    }
    const double *Ex = E, *Ey = E + ng, *Ez = E + 2 * ng;
    const double *By = B, *Bz = B + ng;
    if (r.scheme == kLeapfrog) {
        // B^{n+1/2} into bs first (E* takes its curl), then E* (eq. (EMleapfrog))
        for (int i = threadIdx.x; i < ng; i += nthreads()) {
            b0[i] = lf_bhalf(r, E, B, 0, i);
            b0[tw + i] = lf_bhalf(r, E, B, 1, i);
        }
        lds_barrier();
        for (int i = threadIdx.x; i < ng; i += nthreads()) {
            const int im = i == 0 ? ng - 1 : i - 1;
            e0[i] = Ex[i] - r.hdt * rep_sum(J, i, nrep, rs);
            e0[tw + i] = Ey[i] + r.hdt * (-r.c2 * ((b0[tw + i] - b0[tw + im]) * r.inv_h)
                                          - rep_sum(J, ng + i, nrep, rs));
            e0[2 * tw + i] = Ez[i] + r.hdt * (r.c2 * ((b0[i] - b0[im]) * r.inv_h)
                                              - rep_sum(J, 2 * ng + i, nrep, rs));
        }
        return;
    }
    for (int i = threadIdx.x; i < ng; i += nthreads()) {
        e0[i] = Ex[i] - r.hdt * rep_sum(J, i, nrep, rs);
        e0[tw + i] = Ey[i] + r.hdt * (-r.c2 * dminus(Bz, i, ng, r.inv_h) - rep_sum(J, ng + i, nrep, rs));
        e0[2 * tw + i] = Ez[i] + r.hdt * (r.c2 * dminus(By, i, ng, r.inv_h) - rep_sum(J, 2 * ng + i, nrep, rs));
        b0[i] = By[i] + r.hdt * dplus(Ez, i, ng, r.inv_h);
        b0[tw + i] = Bz[i] - r.hdt * dplus(Ey, i, ng, r.inv_h);
    }
}

// Field update from the centred current J (global): new fields into e1 [ne][ng] and
// b1 [2][ng] (LDS), averaged fields into the interiors of the tiles eb [ne][tw],
// bb [2][tw] (the caller fills the ghosts).  Electromagnetic single runs take these from
// the field launch (k_em_fields) instead; the batched form solves them here.
//   ES: E^{n+1} = E^n - dt (j - mean j)                    (eq. (ampere) in 1D)
//   EM (a = dt/2, s = a^2 c^2, L_h = D-D+), eq. (EMbasic) with Crank-Nicolson:
//     (I - s L_h) E_y' = (I + s L_h) E_y - dt c^2 D-B_z - dt j_y,  B_z' = B_z - a D+(E_y + E_y')
//     (I - s L_h) E_z' = (I + s L_h) E_z + dt c^2 D-B_y - dt j_z,  B_y' = B_y + a D+(E_z + E_z')
//     E_x' = E_x - dt j_x
//   The circulant system is solved with the first row g of its inverse.
// scratch: EM only, 8 N_g doubles of LDS (E^n, B^n, right-hand sides, g).
__device__ __forceinline__ void field_update(const Run &r, const Work &wk, const double *E, const double *B,
                             const double *J, double *e1, double *b1, double *eb, double *bb,
                             double *scratch, double *red, int nrep)
{
    const int ng = r.ng, tw = r.tw, rs = 3 * ng;
    if (r.scheme != 2) {
        // the summed current goes through e1 (each thread rereads its own entries)
        for (int i = threadIdx.x; i < ng; i += nthreads())
            e1[i] = rep_sum(J, i, nrep, rs);
        const double mean = block_mean(e1, ng, red);
        for (int i = threadIdx.x; i < ng; i += nthreads()) {
            const double e0 = E[i];
            const double en = e0 - r.dt * (e1[i] - mean);
            e1[i] = en;
            eb[kGhost + i] = 0.5 * (e0 + en);
        }
        return;
    }
    double *E0 = scratch;            // [3][ng]
    double *B0 = E0 + 3 * ng;        // [2][ng]
    double *R = B0 + 2 * ng;         // [2][ng]
    double *g = R + 2 * ng;          // [ng]
    tile_load(E0, E, 3 * ng);
    tile_load(B0, B, 2 * ng);
    tile_load(g, wk.cninv, ng);
    __syncthreads();
    const double a = r.hdt, s = a * a * r.c2, ih2 = r.inv_h * r.inv_h;
    const double *Ey = E0 + ng, *Ez = E0 + 2 * ng, *By = B0, *Bz = B0 + ng;
    for (int i = threadIdx.x; i < ng; i += nthreads()) {
        const int ip = i + 1 == ng ? 0 : i + 1, im = i == 0 ? ng - 1 : i - 1;
        e1[i] = E0[i] - r.dt * rep_sum(J, i, nrep, rs);
        R[i] = Ey[i] + s * (Ey[ip] - 2.0 * Ey[i] + Ey[im]) * ih2
               - r.dt * r.c2 * dminus(Bz, i, ng, r.inv_h) - r.dt * rep_sum(J, ng + i, nrep, rs);
        R[ng + i] = Ez[i] + s * (Ez[ip] - 2.0 * Ez[i] + Ez[im]) * ih2
                    + r.dt * r.c2 * dminus(By, i, ng, r.inv_h) - r.dt * rep_sum(J, 2 * ng + i, nrep, rs);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ng; i += nthreads()) {
        double ay = 0.0, az = 0.0;
        for (int j = 0; j < ng; ++j) {
            int k = i - j;
            k += k < 0 ? ng : 0;
            ay += g[k] * R[j];
            az += g[k] * R[ng + j];
        }
        e1[ng + i] = ay;
        e1[2 * ng + i] = az;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ng; i += nthreads()) {
        const int ip = i + 1 == ng ? 0 : i + 1;
        b1[ng + i] = Bz[i] - a * ((Ey[ip] + e1[ng + ip]) - (Ey[i] + e1[ng + i])) * r.inv_h;
        b1[i] = By[i] + a * ((Ez[ip] + e1[2 * ng + ip]) - (Ez[i] + e1[2 * ng + i])) * r.inv_h;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * ng; i += nthreads())
        eb[(i / ng) * tw + kGhost + i % ng] = 0.5 * (E0[i] + e1[i]);
    for (int i = threadIdx.x; i < 2 * ng; i += nthreads())
        bb[(i / ng) * tw + kGhost + i % ng] = 0.5 * (B0[i] + b1[i]);
}

// EMEC(LF)'s full step in pass B (eq. (EMleapfrog)), after predictor_fields has put
// B^{n+1/2} into the interior of bs: E^{n+1} = E^n + dt (c^2 curl B^{n+1/2} - j^{*,n+1/2})
// into e1 [3][ng], B^{n+1/2} (the next state's B) into b1 [2][ng], and what v-dagger
// gathers into the interiors of eb ((E^n + E^{n+1})/2) and bb (B^{n+1/2}).
__device__ __forceinline__ void lf_full_fields(const Run &r, const double *E, const double *J,
                                               const double *bs, double *e1, double *b1,
                                               double *eb, double *bb, int nrep)
{
    const int ng = r.ng, tw = r.tw, rs = 3 * ng;
    const double *by = bs + kGhost, *bz = bs + tw + kGhost;
    for (int i = threadIdx.x; i < ng; i += nthreads()) {
        const int im = i == 0 ? ng - 1 : i - 1;
        const double ex = E[i], ey = E[ng + i], ez = E[2 * ng + i];
        const double nx = ex - r.dt * rep_sum(J, i, nrep, rs);
        const double ny = ey + r.dt * (-r.c2 * ((bz[i] - bz[im]) * r.inv_h) - rep_sum(J, ng + i, nrep, rs));
        const double nz = ez + r.dt * (r.c2 * ((by[i] - by[im]) * r.inv_h) - rep_sum(J, 2 * ng + i, nrep, rs));
        e1[i] = nx;
        e1[ng + i] = ny;
        e1[2 * ng + i] = nz;
        eb[kGhost + i] = 0.5 * (ex + nx);
        eb[tw + kGhost + i] = 0.5 * (ey + ny);
        eb[2 * tw + kGhost + i] = 0.5 * (ez + nz);
        b1[i] = by[i];
        b1[ng + i] = bz[i];
        bb[kGhost + i] = by[i];
        bb[tw + kGhost + i] = bz[i];
    }
}

// ESEC2 electrostatic predictor field E* of pass A into the interior of es, exactly as
// predictor_fields computes it, with one round of loads: the replicas of j^{n,*} and E^n
// together (E^n waits in `stash`, ng doubles of LDS that the caller overwrites later).
// Split in two so that the caller can issue its first particle loads in between: load
// completions are counted in order, so loads issued before these would be waited for too.
__device__ __forceinline__ double esec2_predictor_load(const Run &r, const double *E,
                                                       const double *J1, double *es,
                                                       double *stash, int nrep)
{
    const int ng = r.ng, rs = 3 * ng;
    double *e0 = es + kGhost;
    double m = 0.0;
    for (int i = threadIdx.x; i < ng; i += nthreads()) {
        const double en0 = E[i];
        const double a = rep_sum(J1, i, nrep, rs);
        e0[i] = a;
        stash[i] = en0;
        m += a;
    }
    return m;
}

__device__ __forceinline__ void esec2_predictor_finish(const Run &r, double *es,
                                                       const double *stash, double *red, double part)
{
    const int ng = r.ng;
    double *e0 = es + kGhost;
    double m[1] = {part};
    block_reduce<0u>(m, red);
    const double mean = m[0] / ng;
    for (int i = threadIdx.x; i < ng; i += nthreads())
        e0[i] = stash[i] - r.hdt * (e0[i] - mean);
}

// ESEC2 electrostatic fields of pass B: the predictor field E* into the interior of es
// (exactly as predictor_fields computes it), E^{n+1} into e1 and the average into the
// interior of eb (exactly as field_update computes them).  One round of loads (the
// replicas of j^{n,*} and of j^{*,n+1/2}, and E^n, which waits in eb) and one block
// reduction for both means; split in two like esec2_predictor.
struct Sums2 {
    double a, b;
};

__device__ __forceinline__ Sums2 esec2_fields_load(const Run &r, const double *E, const double *J1,
                                                   const double *J2, double *es, double *e1,
                                                   double *eb, int nrep, double *save)
{
    const int ng = r.ng, rs = 3 * ng;
    double *e0 = es + kGhost, *ebi = eb + kGhost;
    Sums2 m = {0.0, 0.0};
    for (int i = threadIdx.x; i < ng; i += nthreads()) {
        const double en0 = E[i];
        const double a = rep_sum(J1, i, nrep, rs);
        const double b = rep_sum(J2, i, nrep, rs);
        e0[i] = a;
        ebi[i] = en0;
        e1[i] = b;
        if (save) {
            save[i] = en0;
            save[ng + i] = a;
            save[2 * ng + i] = b;
        }
        m.a += a;
        m.b += b;
    }
    return m;
}

__device__ __forceinline__ void esec2_fields_finish(const Run &r, double *es, double *e1,
                                                    double *eb, double *red, Sums2 part)
{
    const int ng = r.ng;
    double *e0 = es + kGhost, *ebi = eb + kGhost;
    double m[2] = {part.a, part.b};
    block_reduce<0u>(m, red);
    const double mean1 = m[0] / ng, mean2 = m[1] / ng;
    for (int i = threadIdx.x; i < ng; i += nthreads()) {
        const double en0 = ebi[i];
        e0[i] = en0 - r.hdt * (e0[i] - mean1);
        const double en = en0 - r.dt * (e1[i] - mean2);
        e1[i] = en;
        ebi[i] = 0.5 * (en0 + en);
    }
}

// W_E = h/2 sum |E|^2 and W_B = c^2 h/2 sum |B|^2 (section 5.1) of LDS/global fields;
// every thread gets the result.
__device__ __forceinline__ void field_energies(const Run &r, const double *E, const double *B, double *we,
                               double *wb, double *red)
{
    const bool em = em_scheme(r.scheme);
    const int ng = r.ng, ne = em ? 3 : 1;
    double se = 0.0, sb = 0.0;
    for (int i = threadIdx.x; i < ne * ng; i += nthreads())
        se += E[i] * E[i];
    if (em)
        for (int i = threadIdx.x; i < 2 * ng; i += nthreads())
            sb += B[i] * B[i];
    *we = 0.5 * r.h * block_sum(se, red);
    *wb = em ? 0.5 * r.c2 * r.h * block_sum(sb, red) : 0.0;
}

// Write the record of `step` from the pass-B scalars of every workgroup (summed in a
// fixed order) and the field energies in st; run by one workgroup.
// The standard scheme (Run::scheme == kStandard) has its fields at half steps: its record
// of step n >= 1 is TE at (n - 1/2) dt, the mean of the kinetic energies of steps n - 1
// (slot 4, written by the same pass) and n plus the field energy of E^{n-1/2}.

__device__ __forceinline__ void write_record(const Run &r, const Work &wk, int64_t step, double *red)
{
    const bool half = r.scheme == kStandard && step > 0;
    double ke = 0.0, fb = 0.0, gd = 0.0, nf = 0.0;
    // The kinetic energy is summed by the first wavefront alone (lane l takes workgroups
    // l, l + 64, ... in turn, then the fixed wavefront and workgroup reductions, where the
    // other wavefronts add exact zeros), so the sum does not depend on the size of the
    // workgroup writing the record: a pass and the end-of-call launch write the same
    // record.  The other values are exact (integer sums below 2^53, maxima).
    if (threadIdx.x < 64)
        for (int b = threadIdx.x; b < r.nblocks; b += 64)
            ke += half ? 0.5 * (wk.spart[b * kNS + 0] + wk.spart[b * kNS + 4]) : wk.spart[b * kNS + 0];
    for (int b = threadIdx.x; b < r.nblocks; b += nthreads()) {
        fb += wk.spart[b * kNS + 1];
        gd = fmax(gd, wk.spart[b * kNS + 2]);
        nf = fmax(nf, wk.spart[b * kNS + 3]);
    }
    ke = block_sum(ke, red);
    fb = block_sum(fb, red);
    gd = block_max(gd, red);
    nf = block_max(nf, red);
    if (threadIdx.x == 0) {
        DevState *st = wk.st;
        if (st->flag_a) {
            nf = 1.0;
            st->flag_a = 0;
        }
        if (step == 0) {
            st->fb_total = 0;
            st->nonfinite_sticky = 0;
        }
        const double te = ke + st->we + st->wb;
        if (step == 0)
            st->te0 = te;
        st->fb_total += (int64_t)fb;
        st->nonfinite_sticky |= (nf != 0.0);
        DevRecord rec;
        rec.step = step;
        rec.time = ((double)step - (half ? 0.5 : 0.0)) * r.dt;
        rec.kinetic = ke;
        rec.field_e = st->we;
        rec.field_b = st->wb;
        rec.total = te;
        rec.rel_energy_err = fabs(te - st->te0) / st->te0;
        rec.max_gamma_dev = gd;
        rec.fallbacks = (int64_t)fb;
        rec.fallbacks_total = st->fb_total;
        rec.nonfinite = nf != 0.0;
        rec.pad = 0;
        wk.rec[step % r.rec_cap] = rec;
        st->recorded = step;
    }
}

// --------------------------------------------------------------- particle kernels
template <int NV, bool EM> struct TileSizes {
    static constexpr int ne = EM ? 3 : 1;      // E components gathered
    static constexpr int nb = EM ? 2 : 0;      // B components gathered
    static constexpr int ncur = EM ? 3 : 1;    // current components deposited
};

// The particle's half-step quantities, computed identically in both passes.
template <int ORDER, int NV, bool EM> struct Half {
    double vs[NV];       // v*
    double x1;           // x^{n+1} (unwrapped)
    double xh;           // x^{n+1/2}
};

// Gamma = sqrt(r), r = 1 + rho, rho = num2 / den with num2 = 2 num (eq. (opt_solution));
// r < 0 or a non-finite r (e.g. den = 0) takes the fallback Gamma = 1 and is counted.
// Because Gamma - 1 is tiny for almost every particle (O(dt^4) for ESEC2), the common
// case |rho| < 1e-4 evaluates rho with the hardware reciprocal refined by one Newton step
// (relative error about 2^-46, so below 1e-18 in Gamma) and sqrt(1 + rho) by its Taylor
// series through rho^4 (truncation below 3e-22); any other rho is evaluated with an IEEE
// division and square root.
__device__ __forceinline__ double gamma_factor(double num2, double den, int &fallbacks)
{
    double rc = __builtin_amdgcn_rcp(den);
    rc = fma(rc, fma(-den, rc, 1.0), rc);
    const double rho = num2 * rc;
    if (fabs(rho) < 1e-4)
        return fma(rho, fma(rho, fma(rho, fma(rho, -0.0390625, 0.0625), -0.125), 0.5), 1.0);
    const double rr = 1.0 + num2 / den;
    if (rr >= 0.0 && isfinite(rr))
        return sqrt(rr);
    ++fallbacks;
    return 1.0;
}

// v* solves v* = u + v* x t with u = v^n + dt/2 E**, t = dt/2 B** (eq. (good_translation)
// second line, eq. (EMbasic) fourth line): v* = (u + u x t + (u.t) t) / (1 + |t|^2).
__device__ __forceinline__ void rotate_half(const double u[3], const double t[3], double o[3])
{
    double ut = u[0] * t[0] + u[1] * t[1] + u[2] * t[2];
    double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double inv = 1.0 / (1.0 + tt);
    o[0] = (u[0] + (u[1] * t[2] - u[2] * t[1]) + ut * t[0]) * inv;
    o[1] = (u[1] + (u[2] * t[0] - u[0] * t[2]) + ut * t[1]) * inv;
    o[2] = (u[2] + (u[0] * t[1] - u[1] * t[0]) + ut * t[2]) * inv;
}

// tiles: EM: es[3][tw] predictor E, bs[2][tw] predictor B, ghost-padded; ES: es is the
// coefficient tile of E_x (coef_fill)
template <int ORDER, int NV, bool EM>
__device__ __forceinline__ Half<ORDER, NV, EM> half_step(const Run &r, double x, const double v[NV],
                                                        const double *es, const double *bs)
{
    Half<ORDER, NV, EM> o;
    const double xs = fma(r.hdt, v[0], x);
    if constexpr (NV == 1) {
        o.vs[0] = fma(r.hdt, gather_poly<ORDER>(es, cell_of<ORDER>(xs * r.inv_h - r.xshift, r.ng)), v[0]);
    } else {
        double u[3], t[3];
        if constexpr (EM) {
            const Stencil<ORDER> s = stencil<ORDER>(xs * r.inv_h);
            const Slots<ORDER> n = slots_of<ORDER>(s, r.ng);
            u[0] = fma(r.hdt, gather1<ORDER>(es, s, n), v[0]);
            u[1] = fma(r.hdt, gather1<ORDER>(es + r.tw, s, n), v[1]);
            u[2] = fma(r.hdt, gather1<ORDER>(es + 2 * r.tw, s, n), v[2]);
            const Stencil<ORDER> sh = stencil<ORDER>(xs * r.inv_h - 0.5);
            const Slots<ORDER> nh = slots_of<ORDER>(sh, r.ng);
            t[0] = r.hdt * r.bext[0];
            t[1] = r.hdt * (r.bext[1] + gather1<ORDER>(bs, sh, nh));
            t[2] = r.hdt * (r.bext[2] + gather1<ORDER>(bs + r.tw, sh, nh));
        } else {
            u[0] = fma(r.hdt, gather_poly<ORDER>(es, cell_of<ORDER>(xs * r.inv_h - r.xshift, r.ng)), v[0]);
            u[1] = v[1];
            u[2] = v[2];
            t[0] = r.hdt * r.bext[0];
            t[1] = r.hdt * r.bext[1];
            t[2] = r.hdt * r.bext[2];
        }
        rotate_half(u, t, o.vs);
    }
    o.x1 = fma(r.dt, o.vs[0], x);
    o.xh = 0.5 * (x + o.x1);
    return o;
}

// Pass A of step n (par = n & 1).
// LDS: jt[ncur][tw] | es[ne][tw] | bs[nb][tw]
// pass_a_body processes particles [p0, p1) of one run; `lead` marks the one workgroup
// (per run and launch) that also clears the other predictor current and writes the record.
template <int ORDER, int NV, bool EM, int DEP, int U = kUnrollA<NV>>
__device__ __forceinline__ void pass_a_body(const Run &r, const Work &wk, int par, int64_t step,
                                            const double *__restrict__ X,
                                            const double *__restrict__ V, int64_t p0,
                                            int64_t p1, bool lead, double *smem, double *red,
                                            int *wctr)
{
    using T = TileSizes<NV, EM>;
    const int ng = r.ng, tw = r.tw;
    const unsigned lane = threadIdx.x & 63;
    double *jt = smem;
    double *es = jt + T::ncur * tw;
    double *bs = es + T::ne * tw;
    double *side = bs + T::nb * tw;       // [ncur][tw] FP64 side tile of the deposit
    double *ct = smem + coef_offset((2 * T::ncur + T::ne + T::nb) * tw);   // ES: coefficients
    // pass A walks the state from its end, pass B from its start (see WaveBatches)
    WaveBatches<U> wb(p0, wctr, r.interleave, r.nblocks, r.det, r.np, true);
    PBatch<U, NV> cur, nxt;
    int64_t bcur = wb.first();
    wb.reset();
    if (!EM && r.scheme == 0) {
        const double part = esec2_predictor_load(r, wk.Ef[par], wk.J1[par], es, ct, r.nrep);
        load_batch(cur, X, V, r.vstride, bcur, p1);
        esec2_predictor_finish(r, es, ct, red, part);
    } else if (EM && r.scheme == kPsatd) {
        // E*, B* come from the field launch before this pass
        psatd_tiles(r, wk.ps, es, bs);
        load_batch(cur, X, V, r.vstride, bcur, p1);
    } else {
        predictor_fields(r, wk.Ef[par], EM ? wk.Bf[par] : nullptr, wk.J1[par], es, bs, red, r.nrep);
        load_batch(cur, X, V, r.vstride, bcur, p1);
    }
    tile_zero(jt, T::ncur * tw);
    tile_zero(side, T::ncur * tw);
    // the currents of the next step accumulate into the other buffers (nothing reads them
    // in this pass): every workgroup clears its share
    {
        const int64_t part = p0 / r.chunk, nparts = r.nblocks;
        if (r.scheme != 1)
            rep_zero_part(wk.J1[par ^ 1], T::ncur * ng, r.nrep, 3 * ng, part, nparts);
        rep_zero_part(wk.J2[par ^ 1], T::ncur * ng, r.nrep, 3 * ng, part, nparts);
    }
    // the record of the state this step starts from, if not written yet
    if (lead && step > wk.st->recorded) {
        if (EM && r.scheme == kLeapfrog) {
            const double wbl = lf_magnetic_energy(r, wk.Ef[par], wk.Bf[par], red);
            if (threadIdx.x == 0)
                wk.st->wb = wbl;
        }
        write_record(r, wk, step, red);
    }
    lds_barrier();
    if constexpr (EM) {
        ghost_fill(es, T::ne, ng, tw);
        ghost_fill(bs, T::nb, ng, tw);
    } else {
        coef_fill<ORDER>(ct, es + kGhost, ng, tw);
    }
    lds_barrier();
    const double *eg = EM ? es : ct;     // what half_step gathers E from

    Depo<ORDER, T::ncur, DEP> dep;
    dep.init(side, r, wk.st);
    // whole wavefronts run the loop (DEP = 2 needs them in its deposit); particles past the
    // end are masked with `valid`
    while (bcur < p1) {
        const int64_t bnxt = wb.claim();
        const unsigned nval = (unsigned)min(p1 - bcur, (int64_t)(64 * U));
        double w[U];
        load_weights(w, r.w, r.wu, bcur, p1);
        load_batch(nxt, X, V, r.vstride, bnxt, p1);   // the last one is discarded
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool valid = lane + 64u * u < nval;
            if constexpr (DEP != 2) {
                if (!valid)
                    break;
            }
            const Half<ORDER, NV, EM> hs = half_step<ORDER, NV, EM>(r, cur.x[u], cur.v[u], eg, bs);
            const double q = valid ? w[u] * r.qs : 0.0;
            double qv[T::ncur];
#pragma unroll
            for (int c = 0; c < T::ncur; ++c)
                qv[c] = q * hs.vs[c];
            bool done = false;
            if constexpr (!EM && ORDER == 1 && DEP != 2) {
                if (r.cc) {
                    // exact charge conservation: through the pieces of the path x^n -> x^{n+1}
                    cc_pieces(r, cur.x[u], hs.x1, [&](double base, double t, double f) {
                        double qf[T::ncur];
#pragma unroll
                        for (int c = 0; c < T::ncur; ++c)
                            qf[c] = qv[c] * f;
                        dep.add(jt, tw, ng, cc_stencil(base, t), qf, valid, false);
                    });
                    done = true;
                }
            }
            if (!done)
                dep.add(jt, tw, ng, stencil<ORDER>(hs.xh * r.inv_h), qv, valid, u == 0);
        }
        cur = nxt;
        bcur = bnxt;
    }
    dep.finish(jt, tw, ng);
    flag_over(dep, wk);
    lds_barrier();
    dep.flush_tile(jt, dep_target(r, wk, wk.J2[par]), T::ncur, ng, tw);
}

template <int ORDER, int NV, bool EM, int DEP>
__global__ __launch_bounds__(kMaxThreads<NV>) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<NV>)))
void k_pass_a(Run r, Work wk, int par, int64_t step,
                                                 const double *__restrict__ X,
                                                 const double *__restrict__ V)
{
    extern __shared__ double smem[];
    __shared__ double red[kRedSize];
    __shared__ int wctr;
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    // the lead (which also writes the record) is the last workgroup, whose chunk is the
    // smallest when N_p is not a multiple of it, so its extra work does not lengthen the pass
    pass_a_body<ORDER, NV, EM, DEP>(r, wk, par, step, X, V, p0,
                                    r.interleave ? r.np : min(r.np, p0 + r.chunk),
                                    (int)blockIdx.x == r.nblocks - 1, smem, red, &wctr);
}

// Pass B of step n (par = n & 1): new fields, second gather, Gamma, state write and
// (PRED) the next step's predictor deposit.
// LDS: jt[ncur][tw] | es[ne][tw] | bs[nb][tw] | eb[ne][tw] | bb[nb][tw] | e1[ne][ng] |
//      b1[nb][ng] | EM scratch[8 ng]
// pass_b_body processes particles [p0, p1) of one run and leaves its scalars in
// spart[slot]; `lead` marks the workgroup that publishes the new fields of the run.
template <int ORDER, int NV, bool EM, bool PRED, int DEP, int U = kUnrollB<NV>>
__device__ __forceinline__ void pass_b_body(const Run &r, const Work &wk, int par, const double *X,
                                            const double *V, double *Xo, double *Vo,
                                            int64_t p0, int64_t p1, bool lead, int slot,
                                            double *smem, double *red, int *wctr)
{
    using T = TileSizes<NV, EM>;
    const int ng = r.ng, tw = r.tw;
    const unsigned lane = threadIdx.x & 63;
    WaveBatches<U> wb(p0, wctr, r.interleave, r.nblocks, r.det);
    PBatch<U, NV> cur, nxt;
    int64_t bcur = wb.first();
    wb.reset();
    double *jt = smem;
    double *es = jt + T::ncur * tw;
    double *bs = es + T::ne * tw;
    double *eb = bs + T::nb * tw;
    double *bb = eb + T::ne * tw;
    double *e1 = bb + T::nb * tw;
    double *b1 = e1 + T::ne * ng;
    double *scratch = b1 + T::nb * ng;
    double *side = scratch + (EM ? 8 * ng : 0);   // [ncur][tw] FP64 side tile of the deposit
    // ES: coefficient tiles of E* and E-bar
    double *cts = smem + coef_offset((2 * T::ncur + 2 * T::ne + 2 * T::nb) * tw + (T::ne + T::nb + (EM ? 8 : 0)) * ng);
    double *ctb = cts + (ORDER + 1) * tw;
    const double *En = wk.Ef[par];
    const double *Bn = EM ? wk.Bf[par] : nullptr;
    // the first particle batch is issued after the field loads (see esec2_predictor)
    if (!EM && r.scheme == 0) {
        const Sums2 part = esec2_fields_load(r, En, wk.J1[par], wk.J2[par], es, e1, eb, r.nrep,
                                             lead ? wk.grid_save : nullptr);
        load_batch(cur, X, V, r.vstride, bcur, p1);
        esec2_fields_finish(r, es, e1, eb, red, part);
    } else if (EM && r.em_fields) {
        // the fields v-dagger gathers come from the field launch before this pass, which
        // has also published E^{n+1}, B^{n+1} (the lead reads those back for their
        // energies); E*, B* from the predictor launch (PSATD) or, for the local LI
        // predictor, as in pass A
        if (r.scheme == kPsatd)
            psatd_tiles(r, wk.ps, es, bs);
        else
            predictor_fields(r, En, Bn, wk.J1[par], es, bs, red, r.nrep);
        psatd_tiles(r, wk.pf, eb, bb);
        if (lead) {
            tile_load(e1, wk.Ef[par ^ 1], 3 * ng);
            tile_load(b1, wk.Bf[par ^ 1], 2 * ng);
        }
        load_batch(cur, X, V, r.vstride, bcur, p1);
    } else if (EM && r.scheme == kLeapfrog) {
        predictor_fields(r, En, Bn, wk.J1[par], es, bs, red, r.nrep);
        load_batch(cur, X, V, r.vstride, bcur, p1);
        lf_full_fields(r, En, wk.J2[par], bs, e1, b1, eb, bb, r.nrep);
    } else {
        predictor_fields(r, En, Bn, wk.J1[par], es, bs, red, r.nrep);
        load_batch(cur, X, V, r.vstride, bcur, p1);
        field_update(r, wk, En, Bn, wk.J2[par], e1, b1, eb, bb, scratch, red, r.nrep);
    }
    if constexpr (PRED) {
        tile_zero(jt, T::ncur * tw);
        tile_zero(side, T::ncur * tw);
    }
    lds_barrier();
    if constexpr (EM) {
        ghost_fill(es, T::ne, ng, tw);
        ghost_fill(eb, T::ne, ng, tw);
        ghost_fill(bs, T::nb, ng, tw);
        ghost_fill(bb, T::nb, ng, tw);
    } else {
        coef_fill<ORDER>(cts, es + kGhost, ng, tw);
        coef_fill<ORDER>(ctb, eb + kGhost, ng, tw);
    }
    const double *eg = EM ? es : cts;    // what half_step gathers E* from
    if (lead) {
        // publish E^{n+1} (B^{n+1}) and their energies (pass A clears the next currents)
        if (!(EM && r.em_fields)) {
            for (int i = threadIdx.x; i < T::ne * ng; i += nthreads())
                wk.Ef[par ^ 1][i] = e1[i];
            if constexpr (EM)
                for (int i = threadIdx.x; i < 2 * ng; i += nthreads())
                    wk.Bf[par ^ 1][i] = b1[i];
        }
        if constexpr (!EM) {
            if (wk.grid_save) {
                // the fields this step gathers, for the adjoint's reverse passes
                double *sv = wk.grid_save + 3 * ng;
                for (int i = threadIdx.x; i < ng; i += nthreads()) {
                    sv[i] = es[kGhost + i];
                    sv[ng + i] = eb[kGhost + i];
                    sv[2 * ng + i] = e1[i];
                }
            }
        }
        double we, wb;
        field_energies(r, e1, b1, &we, &wb, red);
        if (threadIdx.x == 0) {
            wk.st->we = we;
            // EMEC(LF)'s W_B needs B^{n+3/2}: the writer of the next record computes it
            if (r.scheme != kLeapfrog)
                wk.st->wb = wb;
        }
    }
    lds_barrier();

    Depo<ORDER, T::ncur, DEP> dep;
    dep.init(side, r, wk.st);
    double ke = 0.0, gdev = 0.0;
    int fb = 0, nonfinite = 0;
    while (bcur < p1) {
        const int64_t bnxt = wb.claim();
        const unsigned nval = (unsigned)min(p1 - bcur, (int64_t)(64 * U));
        double w[U];
        load_weights(w, r.w, r.wu, bcur, p1);
        load_batch(nxt, X, V, r.vstride, bnxt, p1);   // the last one is discarded
        double *Xob = Xo + bcur;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned o = lane + 64u * u;
            const bool valid = o < nval;
            if constexpr (DEP != 2) {
                if (!valid)
                    break;
            }
            const double *v = cur.v[u];
            const Half<ORDER, NV, EM> hs = half_step<ORDER, NV, EM>(r, cur.x[u], v, eg, bs);
            double vd[NV];
            if constexpr (NV == 1) {
                double eb1;
                if constexpr (ORDER == 1)
                    eb1 = r.cc ? cc_gather(r, ctb, cur.x[u], hs.x1)
                               : gather_poly<ORDER>(ctb, cell_of<ORDER>(hs.xh * r.inv_h, ng));
                else
                    eb1 = gather_poly<ORDER>(ctb, cell_of<ORDER>(hs.xh * r.inv_h, ng));
                vd[0] = fma(r.dt, eb1, v[0]);
            } else {
                double e[3], b[3];
                b[0] = r.bext[0];
                if constexpr (EM) {
                    const Stencil<ORDER> s = stencil<ORDER>(hs.xh * r.inv_h);
                    const Slots<ORDER> n = slots_of<ORDER>(s, ng);
                    e[0] = gather1<ORDER>(eb, s, n);
                    e[1] = gather1<ORDER>(eb + tw, s, n);
                    e[2] = gather1<ORDER>(eb + 2 * tw, s, n);
                    const Stencil<ORDER> sh = stencil<ORDER>(hs.xh * r.inv_h - 0.5);
                    const Slots<ORDER> nh = slots_of<ORDER>(sh, ng);
                    b[1] = r.bext[1] + gather1<ORDER>(bb, sh, nh);
                    b[2] = r.bext[2] + gather1<ORDER>(bb + tw, sh, nh);
                } else {
                    if constexpr (ORDER == 1)
                        e[0] = r.cc ? cc_gather(r, ctb, cur.x[u], hs.x1)
                                    : gather_poly<ORDER>(ctb, cell_of<ORDER>(hs.xh * r.inv_h, ng));
                    else
                        e[0] = gather_poly<ORDER>(ctb, cell_of<ORDER>(hs.xh * r.inv_h, ng));
                    e[1] = 0.0;
                    e[2] = 0.0;
                    b[1] = r.bext[1];
                    b[2] = r.bext[2];
                }
                // v-dagger = v^n + dt (E-bar + v* x B-bar)   (eq. (good_translation), (EMbasic))
                vd[0] = v[0] + r.dt * (e[0] + (hs.vs[1] * b[2] - hs.vs[2] * b[1]));
                vd[1] = v[1] + r.dt * (e[1] + (hs.vs[2] * b[0] - hs.vs[0] * b[2]));
                vd[2] = v[2] + r.dt * (e[2] + (hs.vs[0] * b[1] - hs.vs[1] * b[0]));
            }
            // Gamma (eq. (opt_solution)); an imaginary or undefined root falls back to 1.
            // num2 = 2 num = sum (2 v* - (v-dagger + v)) . (v-dagger - v)
            double num2 = 0.0, den = 0.0;
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                const double a2 = fma(2.0, hs.vs[c], -(vd[c] + v[c]));
                num2 = fma(a2, vd[c] - v[c], num2);
                den = fma(vd[c], vd[c], den);
            }
            int fbp = 0;
            const double g = gamma_factor(num2, den, fbp);
            double vn[NV];
            double v2 = 0.0;
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                vn[c] = g * vd[c];
                v2 = fma(vn[c], vn[c], v2);
            }
            const double xw = wrap_pos(hs.x1, r.L);
            const double wp = valid ? w[u] : 0.0;
            if (valid) {
                // the new state is written through to memory (system-scope relaxed stores):
                // nothing in this pass reads it back, and lines left dirty in the L2 of each
                // XCD would be written back at the end of the kernel
#pragma unroll
                for (int c = 0; c < NV; ++c)
                    __hip_atomic_store(&(Vo + c * r.vstride + bcur)[o], vn[c], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&Xob[o], xw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                fb += fbp;
                gdev = fmax(gdev, fabs(g - 1.0));
                ke = fma(wp, v2, ke);
                if (!isfinite(v2) || !isfinite(hs.x1))
                    nonfinite = 1;
            }
            if constexpr (PRED) {
                const double q = wp * r.qs;
                double qv[T::ncur];
#pragma unroll
                for (int c = 0; c < T::ncur; ++c)
                    qv[c] = q * vn[c];
                dep.add(jt, tw, ng, stencil<ORDER>(fma(r.hdt, vn[0], xw) * r.inv_h - r.xshift), qv, valid,
                        u == 0);
            }
        }
        cur = nxt;
        bcur = bnxt;
    }
    if constexpr (PRED) {
        dep.finish(jt, tw, ng);
        nonfinite |= dep.over;
    }
    // kinetic energy and fallbacks (sums), max |Gamma - 1| and the non-finite flag (maxima)
    double sc[4] = {ke, (double)fb, gdev, (double)nonfinite};
    block_reduce<0xcu>(sc, red);
    if (threadIdx.x == 0) {
        wk.spart[slot * kNS + 0] = 0.5 * sc[0];
        wk.spart[slot * kNS + 1] = sc[1];
        wk.spart[slot * kNS + 2] = sc[2];
        wk.spart[slot * kNS + 3] = sc[3];
    }
    if constexpr (PRED) {
        lds_barrier();
        dep.flush_tile(jt, dep_target(r, wk, wk.J1[par ^ 1]), T::ncur, ng, tw);
    }
}

template <int ORDER, int NV, bool EM, bool PRED, int DEP>
__global__ __launch_bounds__(kMaxThreads<NV>) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<NV>)))
void k_pass_b(Run r, Work wk, int par, const double *X,
                                                 const double *V, double *Xo, double *Vo)
{
    extern __shared__ double smem[];
    __shared__ double red[kRedSize];
    __shared__ int wctr;
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    pass_b_body<ORDER, NV, EM, PRED, DEP>(r, wk, par, X, V, Xo, Vo, p0,
                                          r.interleave ? r.np : min(r.np, p0 + r.chunk),
                                          (int)blockIdx.x == r.nblocks - 1, blockIdx.x, smem,
                                          red, &wctr);
}

// ------------------------------------------------------------ ESEC1 in one pass
// ESEC1 (eq. (naivetranslation) with eq. (PICmodification)) has a single grid-wide
// dependency per step: v* uses E^n, which is known before the step, so only the centred
// current j^{n+1/2} -> E^{n+1} needs every particle.  One launch per step therefore
// suffices: it finishes step n (E^{n+1} from j^{n+1/2}, v-dagger, Gamma, the state
// write) and, with x^{n+1}, v^{n+1} still in registers, already computes step n+1's v*
// (gathering the E^{n+1} it has just built) and deposits j^{n+3/2}.  The state is read
// once and written once per step (32 B per particle in 1D-1V).  Step n + 1 recomputes that
// v* from the stored x^{n+1}, v^{n+1} and the stored E^{n+1} with the same instructions,
// so the deposit and the later gather see a bit-identical x^{n+3/2}.  The first step's
// current j^{1/2} is deposited at initialisation by a pass A.
// Currents rotate through three buffers: the pass reads j^{n+1/2} (Jr), deposits
// j^{n+3/2} (Jd) and clears the buffer that held j^{n-1/2} (Jc), which step n + 1 deposits
// into.  The per-workgroup scalars alternate between two arrays as well: this pass's lead
// writes the record of step n from the scalars of the previous pass (wk.spart) while
// the other workgroups write theirs for step n + 1 (spw).
// LDS: jt[ncur][tw] | es[tw] | eb[tw] | e1[ng] | side[ncur][tw] | three coefficient tiles
//      (E^n, E-bar, E^{n+1}), ES only.
template <int ORDER, int NV, int DEP, int U = kUnrollB<NV>>
__device__ __forceinline__ void esec1_body(const Run &r, const Work &wk, int par, int64_t step,
                                           const double *X, const double *V, double *Xo,
                                           double *Vo, const double *Jr, double *Jd, double *Jc,
                                           double *spw, int64_t p0, int64_t p1, bool lead,
                                           int slot, double *smem, double *red, int *wctr)
{
    const int ng = r.ng, tw = r.tw;
    const unsigned lane = threadIdx.x & 63;
    // one pass per step: alternate directions (see WaveBatches)
    WaveBatches<U> wb(p0, wctr, r.interleave, r.nblocks, r.det, r.np, (step & 1) != 0);
    PBatch<U, NV> cur, nxt;
    int64_t bcur = wb.first();
    wb.reset();
    double *jt = smem;
    double *es = jt + tw;
    double *eb = es + tw;
    double *e1 = eb + tw;
    double *side = e1 + ng;
    double *ctn = smem + coef_offset(4 * tw + ng);     // E^n
    double *ctb = ctn + (ORDER + 1) * tw;               // E-bar
    double *ct1 = ctb + (ORDER + 1) * tw;               // E^{n+1}
    const double *En = wk.Ef[par];
    // fields: E^n into es, E^{n+1} into e1, E-bar into eb (field_update, as in pass B)
    for (int i = threadIdx.x; i < ng; i += nthreads())
        es[kGhost + i] = En[i];
    load_batch(cur, X, V, r.vstride, bcur, p1);
    field_update(r, wk, En, nullptr, Jr, e1, nullptr, eb, nullptr, nullptr, red, r.nrep);
    tile_zero(jt, tw);
    tile_zero(side, tw);
    {
        const int64_t part = p0 / r.chunk, nparts = r.nblocks;
        rep_zero_part(Jc, ng, r.nrep, 3 * ng, part, nparts);
    }
    lds_barrier();
    coef_fill<ORDER>(ctn, es + kGhost, ng, tw);
    coef_fill<ORDER>(ctb, eb + kGhost, ng, tw);
    coef_fill<ORDER>(ct1, e1, ng, tw);
    if (lead) {
        // the record of step n (its kinetic energy from the previous pass's scalars, its
        // field energy from st->we), then E^{n+1} and its energy for step n + 1
        if (step > wk.st->recorded)
            write_record(r, wk, step, red);
        for (int i = threadIdx.x; i < ng; i += nthreads())
            wk.Ef[par ^ 1][i] = e1[i];
        double we, wbv;
        field_energies(r, e1, nullptr, &we, &wbv, red);
        if (threadIdx.x == 0) {
            wk.st->we = we;
            wk.st->wb = 0.0;
        }
    }
    lds_barrier();

    Depo<ORDER, 1, DEP> dep;
    dep.init(side, r, wk.st);
    double ke = 0.0, gdev = 0.0;
    int fb = 0, nonfinite = 0;
    while (bcur < p1) {
        const int64_t bnxt = wb.claim();
        const unsigned nval = (unsigned)min(p1 - bcur, (int64_t)(64 * U));
        double w[U];
        load_weights(w, r.w, r.wu, bcur, p1);
        load_batch(nxt, X, V, r.vstride, bnxt, p1);   // the last one is discarded
        double *Xob = Xo + bcur;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned o = lane + 64u * u;
            const bool valid = o < nval;
            if constexpr (DEP != 2) {
                if (!valid)
                    break;
            }
            const double *v = cur.v[u];
            const Half<ORDER, NV, false> hs = half_step<ORDER, NV, false>(r, cur.x[u], v, ctn, nullptr);
            double vd[NV];
            const double eh = gather_poly<ORDER>(ctb, cell_of<ORDER>(hs.xh * r.inv_h, ng));
            if constexpr (NV == 1) {
                vd[0] = fma(r.dt, eh, v[0]);
            } else {
                const double *b = r.bext;
                vd[0] = v[0] + r.dt * (eh + (hs.vs[1] * b[2] - hs.vs[2] * b[1]));
                vd[1] = v[1] + r.dt * (hs.vs[2] * b[0] - hs.vs[0] * b[2]);
                vd[2] = v[2] + r.dt * (hs.vs[0] * b[1] - hs.vs[1] * b[0]);
            }
            double num2 = 0.0, den = 0.0;
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                const double a2 = fma(2.0, hs.vs[c], -(vd[c] + v[c]));
                num2 = fma(a2, vd[c] - v[c], num2);
                den = fma(vd[c], vd[c], den);
            }
            int fbp = 0;
            const double g = gamma_factor(num2, den, fbp);
            double vn[NV];
            double v2 = 0.0;
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                vn[c] = g * vd[c];
                v2 = fma(vn[c], vn[c], v2);
            }
            const double xw = wrap_pos(hs.x1, r.L);
            const double wp = valid ? w[u] : 0.0;
            if (valid) {
#pragma unroll
                for (int c = 0; c < NV; ++c)
                    __hip_atomic_store(&(Vo + c * r.vstride + bcur)[o], vn[c], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&Xob[o], xw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                fb += fbp;
                gdev = fmax(gdev, fabs(g - 1.0));
                ke = fma(wp, v2, ke);
                if (!isfinite(v2) || !isfinite(hs.x1))
                    nonfinite = 1;
            }
            // step n + 1: v* from E^{n+1} at x*_{n+1}, and the centred deposit j^{n+3/2}
            const Half<ORDER, NV, false> h1 = half_step<ORDER, NV, false>(r, xw, vn, ct1, nullptr);
            const double q[1] = {wp * r.qs * h1.vs[0]};
            dep.add(jt, tw, ng, stencil<ORDER>(h1.xh * r.inv_h), q, valid, u == 0);
        }
        cur = nxt;
        bcur = bnxt;
    }
    dep.finish(jt, tw, ng);
    nonfinite |= dep.over;
    double sc[4] = {ke, (double)fb, gdev, (double)nonfinite};
    block_reduce<0xcu>(sc, red);
    if (threadIdx.x == 0) {
        spw[slot * kNS + 0] = 0.5 * sc[0];
        spw[slot * kNS + 1] = sc[1];
        spw[slot * kNS + 2] = sc[2];
        spw[slot * kNS + 3] = sc[3];
    }
    lds_barrier();
    dep.flush_tile(jt, dep_target(r, wk, Jd), 1, ng, tw);
}

template <int ORDER, int NV, int DEP>
__global__ __launch_bounds__(kMaxThreads<NV>) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<NV>)))
void k_esec1(Run r, Work wk, int par, int64_t step, const double *X, const double *V, double *Xo,
             double *Vo, const double *Jr, double *Jd, double *Jc, double *spw)
{
    extern __shared__ double smem[];
    __shared__ double red[kRedSize];
    __shared__ int wctr;
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    esec1_body<ORDER, NV, DEP>(r, wk, par, step, X, V, Xo, Vo, Jr, Jd, Jc, spw, p0,
                               r.interleave ? r.np : min(r.np, p0 + r.chunk),
                               (int)blockIdx.x == r.nblocks - 1, blockIdx.x, smem, red, &wctr);
}

// ------------------------------------------------ standard explicit PIC (comparison)
// The scheme section 5 compares against: Vlasov-Poisson with the leapfrog/Boris push in
// its symmetric form, eq. (symm_Boris): x* = x^n + dt/2 v^n; v^{n+1} = v^n + dt (E^{n+1/2}(x*)
// + v^{n+1/2} x B); x^{n+1} = x* + dt/2 v^{n+1}; E^{n+1/2} is the Gauss field of the charge
// density at the positions x*.  Each step is a field launch (k_std_field: density ->
// E^{n+1/2}) and one particle pass (k_std_pass), which ends by depositing the density at
// x*_{n+1} = x^{n+1} + dt/2 v^{n+1} for the next field launch; the next pass recomputes
// that x* from the stored state with the same instruction.  32 B per particle-step.

// Row of the spectral Gauss solve as a convolution, E_i = sum_j G_{(i - j) mod N} rho_j:
// G_d = (2/N) sum_{m=1}^{M} sin(2 pi m d / N) / k_m, k_m = 2 pi m / L, with M the largest
// mode below the Nyquist mode (the mean and Nyquist modes of E are zero, as in gauss_body).
__device__ void std_green_body(const Run &r, const Work &wk)
{
    const int ng = r.ng;
    for (int d = threadIdx.x; d < ng; d += nthreads()) {
        double acc = 0.0;
        for (int m = 1; 2 * m < ng; ++m) {
            const long long md = ((long long)m * d) % ng;
            const double k = 2.0 * M_PI * m / r.L;
            acc += sinpi(2.0 * (double)md / ng) / k;
        }
        wk.cninv[d] = 2.0 * acc / ng;
    }
}

__global__ __launch_bounds__(1024) void k_std_green(Run r, Work wk) { std_green_body(r, wk); }

// E^{n+1/2} from the density replicas in rho (optionally binomial-filtered once, (1/4,
// 1/2, 1/4)) into E.  A workgroup of 256 threads computes 32 consecutive nodes; for each,
// 8 threads sum consecutive eighths of the convolution in node order and the 8 sums are
// added in order, so the field does not depend on the launch.
// LDS: rho[ng] | g[2 ng] (the Green's row twice, so that (i - j) needs no modulo) |
//      filtered rho[ng].
__global__ __launch_bounds__(256) void k_std_field(Run r, Work wk, const double *rho_rep, double *E,
                                                   int filter)
{
    extern __shared__ double smem[];
    __shared__ double seg[kRedSegments][kRedEntries];
    const int ng = r.ng;
    double *rho = smem, *g = smem + ng, *rf = smem + 3 * ng;
    for (int i = threadIdx.x; i < ng; i += nthreads()) {
        rho[i] = rep_sum(rho_rep, i, r.nrep, 3 * ng);
        const double gi = wk.cninv[i];
        g[i] = gi;
        g[ng + i] = gi;
    }
    __syncthreads();
    if (filter) {
        for (int i = threadIdx.x; i < ng; i += nthreads())
            rf[i] = 0.25 * rho[i == 0 ? ng - 1 : i - 1] + 0.5 * rho[i] + 0.25 * rho[i + 1 == ng ? 0 : i + 1];
        __syncthreads();
        rho = rf;
    }
    const int t = threadIdx.x, e = t % kRedEntries, sg = t / kRedEntries;
    const int i = blockIdx.x * kRedEntries + e;
    const int per = (ng + kRedSegments - 1) / kRedSegments;
    const int j0 = min(ng, sg * per), j1 = min(ng, j0 + per);
    double acc = 0.0;
    if (i < ng)
        for (int j = j0; j < j1; ++j)
            acc = fma(g[i - j + ng], rho[j], acc);
    seg[sg][e] = acc;
    __syncthreads();
    if (sg == 0 && i < ng) {
        double s2 = seg[0][e];
#pragma unroll
        for (int k2 = 1; k2 < kRedSegments; ++k2)
            s2 += seg[k2][e];
        E[i] = s2;
    }
}

// Charge density at x*_0 = x^0 + dt/2 v^0 into J (the first field launch's input).
template <int ORDER>
__device__ __forceinline__ void std_prime_body(const Run &r, const Work &wk,
                                               const double *__restrict__ X,
                                               const double *__restrict__ V, double *J,
                                               int64_t p0, int64_t p1, double *smem)
{
    double *jt = smem;
    double *side = jt + r.tw;
    tile_zero(jt, 2 * r.tw);
    __syncthreads();
    Depo<ORDER, 1, 0> dep;
    dep.init(side, r, wk.st, 1);
    for (int64_t p = p0 + threadIdx.x; p < p1; p += nthreads()) {
        const double q[1] = {(r.w ? r.w[p] : r.wu) * r.qs};
        dep.add(jt, r.tw, r.ng, stencil<ORDER>(fma(r.hdt, V[p], X[p]) * r.inv_h), q);
    }
    flag_over(dep, wk);
    __syncthreads();
    dep.flush_tile(jt, dep_target(r, wk, J), 1, r.ng, r.tw);
}

template <int ORDER>
__global__ __launch_bounds__(1024) void k_std_prime(Run r, Work wk, const double *__restrict__ X,
                                                    const double *__restrict__ V, double *J)
{
    extern __shared__ double smem[];
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    std_prime_body<ORDER>(r, wk, X, V, J, p0, min(r.np, p0 + r.chunk), smem);
}

// One particle pass of step n: gather E^{n+1/2} at x*, the Boris velocity update, the new
// state, the kinetic energies before and after, and the density at x*_{n+1}.
// LDS: jt[tw] | es[tw] | side[tw] | coefficient tile of E^{n+1/2}.
template <int ORDER, int NV, int DEP, int U = kUnrollB<NV>>
__device__ __forceinline__ void std_pass_body(const Run &r, const Work &wk, int par, int64_t step,
                                              const double *X, const double *V, double *Xo,
                                              double *Vo, double *Jd, double *Jc, double *spw,
                                              int64_t p0, int64_t p1, bool lead, int slot,
                                              double *smem, double *red, int *wctr)
{
    const int ng = r.ng, tw = r.tw;
    const unsigned lane = threadIdx.x & 63;
    // one pass per step: alternate directions (see WaveBatches)
    WaveBatches<U> wb(p0, wctr, r.interleave, r.nblocks, r.det, r.np, (step & 1) != 0);
    PBatch<U, NV> cur, nxt;
    int64_t bcur = wb.first();
    wb.reset();
    double *jt = smem;
    double *es = jt + tw;
    double *side = es + tw;
    double *ct = smem + coef_offset(3 * tw);
    const double *Eh = wk.Ef[par];
    for (int i = threadIdx.x; i < ng; i += nthreads())
        es[kGhost + i] = Eh[i];
    load_batch(cur, X, V, r.vstride, bcur, p1);
    tile_zero(jt, tw);
    tile_zero(side, tw);
    {
        const int64_t part = p0 / r.chunk, nparts = r.nblocks;
        rep_zero_part(Jc, ng, r.nrep, 3 * ng, part, nparts);
    }
    lds_barrier();
    coef_fill<ORDER>(ct, es + kGhost, ng, tw);
    if (lead) {
        if (step > wk.st->recorded)
            write_record(r, wk, step, red);
        double we, wbv;
        field_energies(r, es + kGhost, nullptr, &we, &wbv, red);
        if (threadIdx.x == 0) {
            wk.st->we = we;
            wk.st->wb = 0.0;
        }
    }
    lds_barrier();

    Depo<ORDER, 1, DEP> dep;
    dep.init(side, r, wk.st, 1);
    double ke1 = 0.0, ke0 = 0.0;
    int nonfinite = 0;
    while (bcur < p1) {
        const int64_t bnxt = wb.claim();
        const unsigned nval = (unsigned)min(p1 - bcur, (int64_t)(64 * U));
        double w[U];
        load_weights(w, r.w, r.wu, bcur, p1);
        load_batch(nxt, X, V, r.vstride, bnxt, p1);   // the last one is discarded
        double *Xob = Xo + bcur;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned o = lane + 64u * u;
            const bool valid = o < nval;
            if constexpr (DEP != 2) {
                if (!valid)
                    break;
            }
            const double *v = cur.v[u];
            const double xs = fma(r.hdt, v[0], cur.x[u]);
            const double ep = gather_poly<ORDER>(ct, cell_of<ORDER>(xs * r.inv_h, ng));
            double vn[NV];
            if constexpr (NV == 1) {
                vn[0] = fma(r.dt, ep, v[0]);
            } else {
                // v^{n+1/2} = u + v^{n+1/2} x t, u = v^n + dt/2 E, t = dt/2 B; v^{n+1} = 2 v^{n+1/2} - v^n
                const double uu[3] = {fma(r.hdt, ep, v[0]), v[1], v[2]};
                const double tt[3] = {r.hdt * r.bext[0], r.hdt * r.bext[1], r.hdt * r.bext[2]};
                double vh[3];
                rotate_half(uu, tt, vh);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    vn[c] = fma(2.0, vh[c], -v[c]);
            }
            const double x1 = fma(r.hdt, vn[0], xs);
            const double xw = wrap_pos(x1, r.L);
            const double wp = valid ? w[u] : 0.0;
            double v2 = 0.0, v20 = 0.0;
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                v2 = fma(vn[c], vn[c], v2);
                v20 = fma(v[c], v[c], v20);
            }
            if (valid) {
#pragma unroll
                for (int c = 0; c < NV; ++c)
                    __hip_atomic_store(&(Vo + c * r.vstride + bcur)[o], vn[c], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&Xob[o], xw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                ke1 = fma(wp, v2, ke1);
                ke0 = fma(wp, v20, ke0);
                if (!isfinite(v2) || !isfinite(x1))
                    nonfinite = 1;
            }
            // the density of step n + 1 at x*_{n+1}
            const double q[1] = {wp * r.qs};
            dep.add(jt, tw, ng, stencil<ORDER>(fma(r.hdt, vn[0], xw) * r.inv_h), q, valid, u == 0);
        }
        cur = nxt;
        bcur = bnxt;
    }
    dep.finish(jt, tw, ng);
    nonfinite |= dep.over;
    double sc[3] = {ke1, ke0, (double)nonfinite};
    block_reduce<4u>(sc, red);
    if (threadIdx.x == 0) {
        spw[slot * kNS + 0] = 0.5 * sc[0];
        spw[slot * kNS + 1] = 0.0;
        spw[slot * kNS + 2] = 0.0;
        spw[slot * kNS + 3] = sc[2];
        spw[slot * kNS + 4] = 0.5 * sc[1];
    }
    lds_barrier();
    dep.flush_tile(jt, dep_target(r, wk, Jd), 1, ng, tw);
}

template <int ORDER, int NV, int DEP>
__global__ __launch_bounds__(kMaxThreads<NV>) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<NV>)))
void k_std_pass(Run r, Work wk, int par, int64_t step, const double *X, const double *V, double *Xo,
                double *Vo, double *Jd, double *Jc, double *spw)
{
    extern __shared__ double smem[];
    __shared__ double red[kRedSize];
    __shared__ int wctr;
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    std_pass_body<ORDER, NV, DEP>(r, wk, par, step, X, V, Xo, Vo, Jd, Jc, spw, p0,
                                  r.interleave ? r.np : min(r.np, p0 + r.chunk),
                                  (int)blockIdx.x == r.nblocks - 1, blockIdx.x, smem, red, &wctr);
}

// End of a pic_step call (one workgroup): the record of the newest state and a copy of
// the newest fields into the caller's arrays.
__device__ void finish_body(const Run &r, const Work &wk, int par, int64_t step, double *red)
{
    if (step > wk.st->recorded) {
        if (r.scheme == kLeapfrog) {
            const double wbl = lf_magnetic_energy(r, wk.Ef[par], wk.Bf[par], red);
            if (threadIdx.x == 0)
                wk.st->wb = wbl;
        }
        write_record(r, wk, step, red);
    }
    for (int i = threadIdx.x; i < 3 * r.ng; i += nthreads())
        wk.E[i] = wk.Ef[par][i];
    if (em_scheme(r.scheme))
        for (int i = threadIdx.x; i < 2 * r.ng; i += nthreads())
            wk.B[i] = wk.Bf[par][i];
}

__global__ __launch_bounds__(1024) void k_finish(Run r, Work wk, int par, int64_t step)
{
    __shared__ double red[kRedSize];
    finish_body(r, wk, par, step, red);
}

// Copy of the newest record into a caller's device pic_diag (one thread).
__global__ void k_copy_record(Work wk, int rec_cap, DevRecord *dst)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *dst = wk.rec[wk.st->recorded % rec_cap];
}

// ------------------------------------------------------------------- initialisation
// Predictor deposit of the initial state, w v^0 at x*_0 = x^0 + dt/2 v^0, into J1[0].
template <int ORDER, int NV, bool EM>
__device__ __forceinline__ void predeposit_body(const Run &r, const Work &wk,
                                                const double *__restrict__ X,
                                                const double *__restrict__ V, int64_t p0,
                                                int64_t p1, double *smem)
{
    using T = TileSizes<NV, EM>;
    double *jt = smem;
    double *side = jt + T::ncur * r.tw;
    tile_zero(jt, 2 * T::ncur * r.tw);
    __syncthreads();
    Depo<ORDER, T::ncur, 0> dep;
    dep.init(side, r, wk.st);
    for (int64_t p = p0 + threadIdx.x; p < p1; p += nthreads()) {
        const double q = (r.w ? r.w[p] : r.wu) * r.qs;
        double qv[T::ncur];
#pragma unroll
        for (int c = 0; c < T::ncur; ++c)
            qv[c] = q * V[c * r.vstride + p];
        dep.add(jt, r.tw, r.ng, stencil<ORDER>(fma(r.hdt, V[p], X[p]) * r.inv_h - r.xshift), qv);
    }
    flag_over(dep, wk);
    __syncthreads();
    dep.flush_tile(jt, dep_target(r, wk, wk.J1[0]), T::ncur, r.ng, r.tw);
}

template <int ORDER, int NV, bool EM>
__global__ __launch_bounds__(1024) void k_predeposit(Run r, Work wk, const double *__restrict__ X,
                                                     const double *__restrict__ V)
{
    extern __shared__ double smem[];
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    predeposit_body<ORDER, NV, EM>(r, wk, X, V, p0, min(r.np, p0 + r.chunk), smem);
}

// Charge deposit rho_i = (1/h) sum_p w_p S(x_i - x_p) into J2[0] (scratch for Gauss).
template <int ORDER>
__device__ __forceinline__ void deposit_rho_body(const Run &r, const Work &wk,
                                                 const double *__restrict__ X, int64_t p0,
                                                 int64_t p1, double *smem)
{
    double *jt = smem;
    double *side = jt + r.tw;
    tile_zero(jt, 2 * r.tw);
    __syncthreads();
    Depo<ORDER, 1, 0> dep;
    dep.init(side, r, wk.st, 1);
    for (int64_t p = p0 + threadIdx.x; p < p1; p += nthreads()) {
        const double q[1] = {(r.w ? r.w[p] : r.wu) * r.qs};
        dep.add(jt, r.tw, r.ng, stencil<ORDER>(X[p] * r.inv_h), q);
    }
    flag_over(dep, wk);
    __syncthreads();
    dep.flush_tile(jt, dep_target(r, wk, wk.J2[0]), 1, r.ng, r.tw);
}

template <int ORDER>
__global__ __launch_bounds__(1024) void k_deposit_rho(Run r, Work wk, const double *__restrict__ X)
{
    extern __shared__ double smem[];
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    deposit_rho_body<ORDER>(r, wk, X, p0, min(r.np, p0 + r.chunk), smem);
}

// ------------------------------------------------------------- counting-sort rebin
// Particles are reordered by key = kVBins * cell + (v_x >= 0): particles of one cell and
// one direction of motion become contiguous, so a wavefront's particles share a cell or
// two for many steps (gathers become LDS broadcasts, deposits can be summed in registers
// and the global tile flush touches few nodes).  Counting sort: per-workgroup histograms
// (LDS), an exclusive scan of the [key][workgroup] counts, and a scatter in which each
// workgroup places its particles at its own offsets (order inside a key and workgroup is
// unspecified).
__device__ __forceinline__ int sort_key(const Run &r, double x, double vx)
{
    const double cf = floor(x * r.inv_h);
    const int c = (cf >= 0.0 && cf < (double)r.ng) ? (int)cf : (cf >= (double)r.ng ? r.ng - 1 : 0);
    return kVBins * c + (vx >= 0.0 ? 1 : 0);
}

// hist[key * nblocks + b] = number of particles of workgroup b with that key.
__global__ __launch_bounds__(1024) void k_rebin_count(Run r, Work wk, const double *__restrict__ X,
                                                      const double *__restrict__ V)
{
    extern __shared__ int ihist[];
    const int nbins = kVBins * r.ng;
    for (int i = threadIdx.x; i < nbins; i += nthreads())
        ihist[i] = 0;
    __syncthreads();
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    const int64_t p1 = min(r.np, p0 + r.chunk);
    for (int64_t p = p0 + threadIdx.x; p < p1; p += nthreads())
        atomicAdd(&ihist[sort_key(r, X[p], V[p])], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += nthreads())
        wk.hist[(int64_t)i * r.nblocks + blockIdx.x] = ihist[i];
}

// Exclusive scan of hist (length n) in three launches: per-segment sums, a scan of the
// segment sums (one workgroup), and the per-segment rescans.
__global__ __launch_bounds__(1024) void k_scan_sums(const int64_t *a, int64_t n, int64_t seg,
                                                    int64_t *segsum)
{
    __shared__ double red[kRedSize];
    const int64_t s0 = (int64_t)blockIdx.x * seg, s1 = min(n, s0 + seg);
    double acc = 0.0;     // counts are exact in double below 2^53
    for (int64_t i = s0 + threadIdx.x; i < s1; i += nthreads())
        acc += (double)a[i];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0)
        segsum[blockIdx.x] = (int64_t)acc;
}

__global__ __launch_bounds__(1024) void k_scan_top(int64_t *segsum, int nseg)
{
    // nseg <= blockDim: one value per thread, Hillis-Steele in LDS
    __shared__ int64_t buf[1024];
    const int t = threadIdx.x;
    const int64_t mine = t < nseg ? segsum[t] : 0;
    buf[t] = mine;
    __syncthreads();
    for (int off = 1; off < (int)nthreads(); off <<= 1) {
        const int64_t add = t >= off ? buf[t - off] : 0;
        __syncthreads();
        buf[t] += add;
        __syncthreads();
    }
    if (t < nseg)
        segsum[t] = buf[t] - mine;     // exclusive
}

__global__ __launch_bounds__(1024) void k_scan_apply(int64_t *a, int64_t n, int64_t seg,
                                                     const int64_t *segsum)
{
    // in-place exclusive scan of one segment, processed in chunks of blockDim elements
    __shared__ int64_t buf[1024];
    const int t = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * seg, s1 = min(n, s0 + seg);
    int64_t carry = segsum[blockIdx.x];
    for (int64_t c0 = s0; c0 < s1; c0 += nthreads()) {
        const int64_t i = c0 + t;
        const int64_t mine = i < s1 ? a[i] : 0;
        buf[t] = mine;
        __syncthreads();
        for (int off = 1; off < (int)nthreads(); off <<= 1) {
            const int64_t add = t >= off ? buf[t - off] : 0;
            __syncthreads();
            buf[t] += add;
            __syncthreads();
        }
        if (i < s1)
            a[i] = carry + buf[t] - mine;
        const int64_t total = buf[nthreads() - 1];
        __syncthreads();
        carry += total;
    }
}

// Scatter the state (and ids, weights) of each workgroup's particles to their sorted
// positions in the second buffers.
template <int NV>
__global__ __launch_bounds__(1024) void k_rebin_scatter(Run r, Work wk, const double *__restrict__ X,
                                                        const double *__restrict__ V,
                                                        const int64_t *__restrict__ ID)
{
    extern __shared__ int64_t cursor[];
    const int nbins = kVBins * r.ng;
    for (int i = threadIdx.x; i < nbins; i += nthreads())
        cursor[i] = wk.hist[(int64_t)i * r.nblocks + blockIdx.x];
    __syncthreads();
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    const int64_t p1 = min(r.np, p0 + r.chunk);
    for (int64_t p = p0 + threadIdx.x; p < p1; p += nthreads()) {
        const double x = X[p];
        const int key = sort_key(r, x, V[p]);
        const int64_t d = (int64_t)atomicAdd((unsigned long long *)&cursor[key], 1ull);
        wk.x2[d] = x;
#pragma unroll
        for (int c = 0; c < NV; ++c)
            wk.v2[c * r.np + d] = V[c * r.vstride + p];
        if (ID)
            wk.id2[d] = ID[p];
        if (wk.wcur)
            wk.w2[d] = wk.wcur[p];
    }
}

__global__ void k_copy_i64(int64_t *dst, const int64_t *src, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * nthreads() + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * nthreads())
        dst[i] = src[i];
}

__global__ void k_copy_f64(double *dst, const double *src, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * nthreads() + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * nthreads())
        dst[i] = src[i];
}

// Wrap positions into [0, L); the initial kinetic energy and non-finite flag go to
// spart[slot] like the scalars of a pass B.
template <int NV>
__device__ __forceinline__ void init_particles_body(const Run &r, const Work &wk,
                                                    double *__restrict__ X,
                                                    const double *__restrict__ V, int64_t p0,
                                                    int64_t p1, int slot, double *red)
{
    double ke = 0.0, ws = 0.0, wmax = 0.0, wvmax = 0.0;
    int nonfinite = 0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += nthreads()) {
        double v2 = 0.0, vm = 0.0;
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            const double vc = V[c * r.vstride + p];
            v2 += vc * vc;
            vm = fmax(vm, fabs(vc));
        }
        const double x = X[p];
        if (!isfinite(x) || !isfinite(v2))
            nonfinite = 1;
        X[p] = wrap_pos(x, r.L);
        const double wp = r.w ? r.w[p] : r.wu;
        ke += wp * v2;
        ws += wp;
        wmax = fmax(wmax, fabs(wp));
        wvmax = fmax(wvmax, fabs(wp) * vm);
    }
    double sums[2] = {ke, ws}, maxes[3] = {(double)nonfinite, wmax, wvmax};
    block_reduce<0u>(sums, red);
    block_reduce<7u>(maxes, red);
    if (threadIdx.x == 0) {
        wk.spart[slot * kNS + 0] = 0.5 * sums[0];
        wk.spart[slot * kNS + 1] = 0.0;
        wk.spart[slot * kNS + 2] = 0.0;
        wk.spart[slot * kNS + 3] = maxes[0];
        wk.spart[slot * kNS + 4] = sums[1];
        wk.spart[slot * kNS + 5] = maxes[1];
        wk.spart[slot * kNS + 6] = maxes[2];
    }
}

template <int NV>
__global__ __launch_bounds__(1024) void k_init_particles(Run r, Work wk, double *__restrict__ X,
                                                         const double *__restrict__ V)
{
    __shared__ double red[kRedSize];
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    init_particles_body<NV>(r, wk, X, V, p0, min(r.np, p0 + r.chunk), blockIdx.x, red);
}

// Fixed-point scales of the deposit tiles (one workgroup per run), from the initial
// particles' slots 4-6: the charge density's from the largest weight (a charge
// contribution is at most w / h), the currents' from twice the largest w |v| (or w, if
// that is larger: speeds are in thermal units).  2^S is the largest power of two with
// q 2^S <= Run::fx_lim for that reference contribution q.
__device__ void fx_setup_body(const Run &r, const Work &wk, double *red)
{
    double wmax = 0.0, wvmax = 0.0;
    for (int b = threadIdx.x; b < r.nblocks; b += nthreads()) {
        wmax = fmax(wmax, wk.spart[b * kNS + 5]);
        wvmax = fmax(wvmax, wk.spart[b * kNS + 6]);
    }
    double m[2] = {wmax, wvmax};
    block_reduce<3u>(m, red);
    if (threadIdx.x == 0) {
        const double qref[2] = {2.0 * fmax(m[1], m[0]) * r.inv_h, m[0] * r.inv_h};
        for (int k = 0; k < 2; ++k) {
            int S = 0;
            if (qref[k] > 0.0 && isfinite(qref[k]))
                S = (int)floor(log2(r.fx_lim / qref[k]));
            S = max(-1000, min(1000, S));
            wk.st->fx_scale[k] = ldexp(1.0, S);
            wk.st->fx_inv[k] = ldexp(1.0, -S);
        }
        wk.st->flag_a = 0;
    }
}

__global__ __launch_bounds__(1024) void k_fx_setup(Run r, Work wk)
{
    __shared__ double red[kRedSize];
    fx_setup_body(r, wk, red);
}

// Deterministic mode: J[c][i] = the sum over the workgroups b of part[b][c][i] (replica 0
// of a current; the deterministic mode keeps one replica), always in the same order: a
// workgroup of 256 threads takes 32 consecutive entries; for each entry, 8 threads sum
// consecutive eighths of the rows in row order, and the 8 sums are then added in order.

__global__ __launch_bounds__(256) void k_reduce_partials(const double *__restrict__ part,
                                                         double *__restrict__ J, int nblocks,
                                                         int n, int rowlen)
{
    __shared__ double seg[kRedSegments][kRedEntries];
    const int t = threadIdx.x, e = t % kRedEntries, sg = t / kRedEntries;
    const int idx = blockIdx.x * kRedEntries + e;
    const int per = (nblocks + kRedSegments - 1) / kRedSegments;
    const int b0 = min(nblocks, sg * per), b1 = min(nblocks, b0 + per);
    double acc = 0.0;
    if (idx < n) {
        int b = b0;
        for (; b + 8 <= b1; b += 8) {
            double v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                v[k] = part[(size_t)(b + k) * rowlen + idx];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                acc += v[k];
        }
        for (; b < b1; ++b)
            acc += part[(size_t)b * rowlen + idx];
    }
    seg[sg][e] = acc;
    __syncthreads();
    if (sg == 0 && idx < n) {
        double s = seg[0][e];
#pragma unroll
        for (int k = 1; k < kRedSegments; ++k)
            s += seg[k][e];
        J[idx] = s;
    }
}

// Initial Gauss solve: dE/dx = rho - 1 with rho in J2[0], into the caller's E_x.
// Spectrally on the nodes: E_m = rho_m / (i k_m), k_m = 2 pi m / L for 0 < |m| < N/2, mean
// and Nyquist modes zero (the Poisson form, eq. (poisson), in 1D).
// LDS: rho | Re E_m | Im E_m | the cosines and sines of 2 pi j / N_g, computed once by the
// same calls the sums would make term by term (the sums index them with m l mod N_g), so
// the result is the same bit for bit (5 N_g doubles: every grid the passes accept fits).
__host__ __device__ constexpr size_t gauss_lds_doubles(int ng)
{
    return 5 * (size_t)ng;
}

__device__ void gauss_body(const Run &r, const Work &wk, double *smem)
{
    const int ng = r.ng;
    double *rho = smem, *er = smem + ng, *ei = smem + 2 * ng;
    double *tc = smem + 3 * ng, *ts = smem + 4 * ng;
    rep_gather(rho, wk.J2[0], ng, r.nrep, 3 * ng);
    for (int j = threadIdx.x; j < ng; j += nthreads())
        sincospi(2.0 * (double)j / ng, &ts[j], &tc[j]);
    __syncthreads();
    if (r.filter_rho) {
        // the standard scheme's filtered density (as in k_std_field), through ei
        for (int i = threadIdx.x; i < ng; i += nthreads())
            ei[i] = 0.25 * rho[i == 0 ? ng - 1 : i - 1] + 0.5 * rho[i] + 0.25 * rho[i + 1 == ng ? 0 : i + 1];
        __syncthreads();
        for (int i = threadIdx.x; i < ng; i += nthreads())
            rho[i] = ei[i];
        __syncthreads();
    }
    for (int m = threadIdx.x; m < ng; m += nthreads()) {
        double re = 0.0, im = 0.0;
        if (m != 0 && 2 * m != ng) {
            int ml = 0;                        // m l mod N_g
            for (int l = 0; l < ng; ++l) {
                re += rho[l] * tc[ml];
                im -= rho[l] * ts[ml];
                ml += m;
                ml -= ml >= ng ? ng : 0;
            }
            const int ms = m <= ng / 2 ? m : m - ng;
            const double k = 2.0 * M_PI * ms / r.L;
            const double tr = re, ti = im;
            re = ti / k;          // (tr + i ti) / (i k) = ti / k - i tr / k
            im = -tr / k;
        }
        er[m] = re;
        ei[m] = im;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ng; i += nthreads()) {
        double acc = 0.0;
        int mi = i;                            // m i mod N_g, from m = 1
        for (int m = 1; m < ng; ++m) {
            acc += er[m] * tc[mi] - ei[m] * ts[mi];
            mi += i;
            mi -= mi >= ng ? ng : 0;
        }
        wk.E[i] = acc / ng;
    }
}

__global__ __launch_bounds__(1024) void k_gauss(Run r, Work wk)
{
    extern __shared__ double smem[];
    gauss_body(r, wk, smem);
}

// Initial field of a charge-conserving run (Run::cc): Gauss' law on the half-node E,
// (E_{i+1/2} - E_{i-1/2}) / h = rho_i - mean(rho), by a running sum from the density in
// J2[0] (quadratic B-spline on the nodes), then the mean of E removed (E = -d(phi)/dx).
// One workgroup; the running sum is serial (N_g additions).
__global__ __launch_bounds__(1024) void k_gauss_cc(Run r, Work wk)
{
    extern __shared__ double smem[];
    __shared__ double red[kRedSize];
    const int ng = r.ng;
    double *rho = smem;
    rep_gather(rho, wk.J2[0], ng, r.nrep, 3 * ng);
    __syncthreads();
    const double m = block_mean(rho, ng, red);
    if (threadIdx.x == 0) {
        double e = 0.0;
        rho[0] = 0.0;               // rho[i] now holds E_{i+1/2}
        for (int i = 1; i < ng; ++i) {
            e += r.h * (rho[i] - m);
            rho[i] = e;
        }
    }
    __syncthreads();
    const double me = block_mean(rho, ng, red);
    for (int i = threadIdx.x; i < ng; i += nthreads())
        wk.E[i] = rho[i] - me;
}

// First row of (I - s L_h)^{-1} for the periodic 3-point Laplacian: circulant, so
// g_k = (1/N) sum_m cos(2 pi m k / N) / (1 + s (4/h^2) sin^2(pi m / N)).  Used by the
// batched form, whose pass B solves Crank-Nicolson in its prologue (field_update).
__device__ void cn_init_body(const Run &r, const Work &wk)
{
    const int ng = r.ng;
    const double s = r.hdt * r.hdt * r.c2;
    for (int k = threadIdx.x; k < ng; k += nthreads()) {
        double acc = 0.0;
        for (int m = 0; m < ng; ++m) {
            const double sn = sinpi((double)m / ng);
            const double lam = 1.0 + s * 4.0 * r.inv_h * r.inv_h * sn * sn;
            const long long mk = ((long long)m * k) % ng;
            acc += cospi(2.0 * (double)mk / ng) / lam;
        }
        wk.cninv[k] = acc / ng;
    }
}


// ------------------------------------------------------------------- EMEC(PSATD)
// Field updates of the electromagnetic schemes as real-space convolutions.
// EMEC(PSATD) (section 4.2): the semi-discrete Maxwell system with the
// current held fixed, dE/dt = c^2 curl B - j, dB/dt = -curl E, integrated exactly over a
// time tau for each Fourier mode (eq. (PSATDformula)), and the time average of E over the
// step (its time integral).  In 1D the transverse pairs (E_y, B_z) and (E_z, -B_y) both
// obey dE/dt = -c^2 D- B - j, dB/dt = -D+ E with E, j on the nodes and B on the half
// nodes; the curls are spectral on this staggered grid: D+ (nodes to half nodes)
// multiplies mode k by a = i k e^{i k h/2}, D- (half nodes to nodes) by
// b = i k e^{-i k h/2}, so that a b = -k^2.  With w = c |k|, C = cos(w tau),
// S = sin(w tau) and 1 - C = 2 sin^2(w tau / 2):
//   E(tau) = C E - c^2 b S/w B - S/w j,   B(tau) = C B - a S/w E + a (1 - C)/w^2 j,
//   <E>    = S/(w tau) E - c^2 b (1 - C)/(w^2 tau) B - (1 - C)/(w^2 tau) j,
// and mode 0: E - tau j, B, E - tau/2 j.  Each map is a circulant convolution in real
// space, out_i = sum_j K[(i - j) mod N] in_j, whose row K[d] = (1/N) Re sum_m K(m)
// e^{2 pi i m d / N} (m signed, |m| <= N/2; every symbol is real at the Nyquist mode)
// is computed once here: grid (ceil(N / blockDim), kPsatdRows).
__device__ __forceinline__ void psatd_symbol(const Run &r, int row, int ms, double &sr, double &si)
{
    const bool full = row >= kRowC2;
    const double tau = full ? r.dt : r.hdt;
    if (ms == 0) {
        sr = (row == kRowC1 || row == kRowC2 || row == kRowAE) ? 1.0
             : (row == kRowEJ1 || row == kRowEJ2) ? -tau
             : row == kRowAJ ? -0.5 * tau : 0.0;
        si = 0.0;
        return;
    }
    const double k = 2.0 * M_PI * (double)ms / r.L;
    const double w = sqrt(r.c2) * fabs(k);
    double sh, ch;                       // e^{i k h/2} = ch + i sh, k h/2 = pi ms / N
    sincospi((double)ms / r.ng, &sh, &ch);
    double S, C;
    sincos(w * tau, &S, &C);
    const double sh2 = sin(0.5 * w * tau);
    const double omc = 2.0 * sh2 * sh2;  // 1 - C
    // a = i k e^{i k h/2} = k (-sh + i ch),  b = i k e^{-i k h/2} = k (sh + i ch)
    switch (row) {
    case kRowC1: case kRowC2: sr = C; si = 0.0; break;
    case kRowEB1: case kRowEB2: sr = -r.c2 * S / w * k * sh; si = -r.c2 * S / w * k * ch; break;
    case kRowEJ1: case kRowEJ2: sr = -S / w; si = 0.0; break;
    case kRowBE1: case kRowBE2: sr = S / w * k * sh; si = -S / w * k * ch; break;
    case kRowBJ1: case kRowBJ2: sr = -omc / (w * w) * k * sh; si = omc / (w * w) * k * ch; break;
    case kRowAE: sr = S / (w * tau); si = 0.0; break;
    case kRowAB: sr = -r.c2 * omc / (w * w * tau) * k * sh; si = -r.c2 * omc / (w * w * tau) * k * ch; break;
    default: sr = -omc / (w * w * tau); si = 0.0; break;   // kRowAJ
    }
}

// The same rows for EMEC(LI) (eq. (EMbasic) with Crank-Nicolson), from the symbols of the
// staggered differences, D+ -> a = (e^{i k h} - 1)/h and D- -> b = (1 - e^{-i k h})/h, with
// lambda = s a b = -4 s sin^2(k h/2)/h^2 (s = (dt/2)^2 c^2) and d = 1 - lambda:
//   predictor (explicit half step): E* = E - dt/2 c^2 b B - dt/2 j, B* = B - dt/2 a E;
//   full step: E' = (1 + lambda)/d E - dt c^2 b/d B - dt/d j,
//              B' = B - dt/2 a (E + E') = (1 + lambda)/d B - dt a/d E + dt^2 a/(2 d) j;
//   average (E + E')/2 = E/d - dt c^2 b/(2 d) B - dt/(2 d) j.
__device__ __forceinline__ void cn_symbol(const Run &r, int row, int ms, double &sr, double &si)
{
    double st, ct, sh;                   // sin, cos of k h = 2 pi ms / N; sin(k h/2)
    sincospi(2.0 * (double)ms / r.ng, &st, &ct);
    sh = sinpi((double)ms / r.ng);
    const double omc = 2.0 * sh * sh;    // 1 - cos(k h)
    // a = (-omc + i st)/h,  b = (omc + i st)/h
    const double ar = -omc * r.inv_h, ai = st * r.inv_h, br = omc * r.inv_h, bi = st * r.inv_h;
    const double s = r.hdt * r.hdt * r.c2;
    const double lam = -4.0 * s * sh * sh * r.inv_h * r.inv_h, d = 1.0 - lam;
    const double dt = r.dt;
    switch (row) {
    case kRowC1: sr = 1.0; si = 0.0; break;
    case kRowEB1: sr = -r.hdt * r.c2 * br; si = -r.hdt * r.c2 * bi; break;
    case kRowEJ1: sr = -r.hdt; si = 0.0; break;
    case kRowBE1: sr = -r.hdt * ar; si = -r.hdt * ai; break;
    case kRowBJ1: sr = 0.0; si = 0.0; break;
    case kRowC2: sr = (1.0 + lam) / d; si = 0.0; break;
    case kRowEB2: sr = -dt * r.c2 * br / d; si = -dt * r.c2 * bi / d; break;
    case kRowEJ2: sr = -dt / d; si = 0.0; break;
    case kRowBE2: sr = -dt * ar / d; si = -dt * ai / d; break;
    case kRowBJ2: sr = dt * dt * ar / (2.0 * d); si = dt * dt * ai / (2.0 * d); break;
    case kRowAE: sr = 1.0 / d; si = 0.0; break;
    case kRowAB: sr = -dt * r.c2 * br / (2.0 * d); si = -dt * r.c2 * bi / (2.0 * d); break;
    default: sr = -dt / (2.0 * d); si = 0.0; break;   // kRowAJ
    }
}

// Rows of the electromagnetic field updates (EMEC(PSATD) or EMEC(LI) by Run::scheme):
// grid (ceil(N / blockDim), kPsatdRows).
__global__ __launch_bounds__(256) void k_em_rows(Run r, Work wk)
{
    extern __shared__ double sym[];      // [2][ng]: the row's symbol, real and imaginary
    const int ng = r.ng, row = blockIdx.y;
    for (int m = threadIdx.x; m < ng; m += nthreads()) {
        const int ms = 2 * m <= ng ? m : m - ng;
        if (r.scheme == kPsatd)
            psatd_symbol(r, row, ms, sym[m], sym[ng + m]);
        else
            cn_symbol(r, row, ms, sym[m], sym[ng + m]);
    }
    __syncthreads();
    const int d = blockIdx.x * nthreads() + threadIdx.x;
    if (d >= ng)
        return;
    double acc = 0.0;
    for (int m = 0; m < ng; ++m) {
        double sn, cs;
        const long long q = ((long long)m * d) % ng;
        sincospi(2.0 * (double)q / ng, &sn, &cs);
        acc += sym[m] * cs - sym[ng + m] * sn;
    }
    wk.prow[(size_t)row * ng + d] = acc / ng;
}

// One electromagnetic field update by the rows of k_em_rows.  full = 0: the predictor
// fields (E*, B*) into ps (EMEC(PSATD): PSATD(E^n, B^n, j^{n,*}, dt/2), eq. (EM_PSATD)
// second line); full = 1: (E^{n+1}, B^{n+1}) from E^n, B^n and j^{*,n+1/2} into
// Ef[par ^ 1], Bf[par ^ 1], and into pf the E that v-dagger gathers (PSATD: the time
// average <E> over the step; LI: (E^n + E^{n+1})/2) and B^{n+1/2} = (B^n + B^{n+1})/2.
// Grid (ceil(N / kPsatdOut), nq), 256 threads: blockIdx.y picks the pair p and the output
// o (predictor: q = 2 p + o, o = E, B; full: q = 3 p + o, o = E, B, <E>); a workgroup
// computes kPsatdOut nodes, each as kPsatdSeg partial sums over consecutive ranges of j
// (in increasing j) added in segment order, so the update is reproducible.  E_x has no
// curl term: E_x - tau j_x (average E_x - tau/2 j_x), written by q = 0.
// LDS: e | B (signed) | j | the three rows [6][N] | partial sums [kPsatdSeg][kPsatdOut].
constexpr int kPsatdOut = 32, kPsatdSeg = 8;

__global__ __launch_bounds__(256) void k_em_fields(Run r, Work wk, int par, int full)
{
    extern __shared__ double sm[];
    const int ng = r.ng, rs = 3 * ng, q = blockIdx.y;
    const int p = full ? q / 3 : q >> 1, o = full ? q % 3 : q & 1;
    const double *E = wk.Ef[par], *B = wk.Bf[par], *J = full ? wk.J2[par] : wk.J1[par];
    const int bc = p == 0 ? 1 : 0;       // pair 0: B_z, pair 1: B_y (taken as -B_y)
    const double sg = p == 0 ? 1.0 : -1.0;
    double *e = sm, *b = sm + ng, *jj = sm + 2 * ng, *k0 = sm + 3 * ng, *k1 = sm + 4 * ng,
           *k2 = sm + 5 * ng, *part = sm + 6 * ng;
    int r0, r1, r2;
    if (o == 0) {
        r0 = full ? kRowC2 : kRowC1; r1 = full ? kRowEB2 : kRowEB1; r2 = full ? kRowEJ2 : kRowEJ1;
    } else if (o == 1) {
        r0 = full ? kRowBE2 : kRowBE1; r1 = full ? kRowC2 : kRowC1; r2 = full ? kRowBJ2 : kRowBJ1;
    } else {
        r0 = kRowAE; r1 = kRowAB; r2 = kRowAJ;
    }
    for (int i = threadIdx.x; i < ng; i += nthreads()) {
        e[i] = E[(1 + p) * ng + i];
        b[i] = sg * B[bc * ng + i];
        jj[i] = rep_sum(J, (1 + p) * ng + i, r.nrep, rs);
        k0[i] = wk.prow[(size_t)r0 * ng + i];
        k1[i] = wk.prow[(size_t)r1 * ng + i];
        k2[i] = wk.prow[(size_t)r2 * ng + i];
    }
    __syncthreads();
    const int il = threadIdx.x % kPsatdOut, seg = threadIdx.x / kPsatdOut;
    const int i = blockIdx.x * kPsatdOut + il;
    const int len = (ng + kPsatdSeg - 1) / kPsatdSeg;
    const int j0 = seg * len, j1 = min(ng, j0 + len);
    double acc = 0.0;
    if (i < ng) {
        int k = i - j0;
        k += k < 0 ? ng : 0;
        for (int j = j0; j < j1; ++j) {
            acc = fma(k0[k], e[j], acc);
            acc = fma(k1[k], b[j], acc);
            acc = fma(k2[k], jj[j], acc);
            k = k == 0 ? ng - 1 : k - 1;
        }
    }
    part[seg * kPsatdOut + il] = acc;
    __syncthreads();
    if (seg != 0 || i >= ng)
        return;
    acc = part[il];
    for (int t = 1; t < kPsatdSeg; ++t)
        acc += part[t * kPsatdOut + il];
    if (!full) {
        if (o == 0)
            wk.ps[(1 + p) * ng + i] = acc;
        else
            wk.ps[(3 + bc) * ng + i] = sg * acc;
    } else if (o == 0) {
        wk.Ef[par ^ 1][(1 + p) * ng + i] = acc;
    } else if (o == 1) {
        const double bn = sg * acc;
        wk.Bf[par ^ 1][bc * ng + i] = bn;
        wk.pf[(3 + bc) * ng + i] = 0.5 * (B[bc * ng + i] + bn);
    } else {
        wk.pf[(1 + p) * ng + i] = acc;
    }
    if (q == 0) {
        const double ex = E[i], jx = rep_sum(J, i, r.nrep, rs);
        if (full) {
            wk.Ef[par ^ 1][i] = ex - r.dt * jx;
            wk.pf[i] = ex - r.hdt * jx;
        } else {
            wk.ps[i] = ex - r.hdt * jx;
        }
    }
}


// Initial fields into the parity-0 buffers and the record of step 0 (one workgroup).
__device__ void init_finish_body(const Run &r, const Work &wk, double *red)
{
    const int ng = r.ng;
    for (int i = threadIdx.x; i < 3 * ng; i += nthreads())
        wk.Ef[0][i] = wk.E[i];
    if (em_scheme(r.scheme))
        for (int i = threadIdx.x; i < 2 * ng; i += nthreads())
            wk.Bf[0][i] = wk.B[i];
    double we, wb;
    field_energies(r, wk.E, wk.B, &we, &wb, red);
    if (r.scheme == kLeapfrog)
        wb = lf_magnetic_energy(r, wk.E, wk.B, red);
    if (threadIdx.x == 0) {
        wk.st->we = we;
        wk.st->wb = wb;
        wk.st->recorded = -1;
    }
    // the charge scratch must be zero before the first centred deposit
    rep_zero(wk.J2[0], 3 * ng, r.nrep, 3 * ng);
    __syncthreads();
    write_record(r, wk, 0, red);
}

__global__ __launch_bounds__(1024) void k_init_finish(Run r, Work wk)
{
    __shared__ double red[kRedSize];
    init_finish_body(r, wk, red);
}

__global__ void k_fill(double *p, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * nthreads() + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * nthreads())
        p[i] = v;
}

// ----------------------------------------------------------------- batched ensemble
// Many independent runs (different N_p, N_g, L) advanced together.  Particles of all
// runs are packed in one structure of arrays; each run keeps its own fields, currents,
// state and records.  The work is a table of items, each a chunk of one run's
// particles (chunks of a run are consecutive; the first is the run's lead).  Every pass
// is ONE launch of a persistent grid whose workgroups stride over the table, so runs of
// very different sizes load-balance; the step number is read from a device counter so
// that a captured graph of several steps can be replayed unchanged.
struct BatchRun {
    Run r;                 // scalars; r.nblocks = items of this run, r.vstride = packed N
    Work wk;               // this run's arrays (spart points at its first item's slot)
    int64_t poff;          // first particle of the run in the packed arrays
};

struct BatchItem {
    int32_t run;
    int32_t slot;          // chunk index within the run (0 = lead)
    int64_t p0, p1;        // run-local particle range
};

// Copy of a structure that is the same for the whole workgroup (a run's scalars and
// arrays) into scalar registers, one 32-bit word at a time.
template <int N> struct Words {
    int w[N];
};

template <typename T> __device__ __forceinline__ T uniform_copy(const T &g)
{
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    constexpr int n = (int)(sizeof(T) / 4);
    Words<n> w = __builtin_bit_cast(Words<n>, g);
#pragma unroll
    for (int i = 0; i < n; ++i)
        w.w[i] = __builtin_amdgcn_readfirstlane(w.w[i]);
    return __builtin_bit_cast(T, w);
}

// A structure that no thread writes during the kernel and that the whole workgroup reads
// at one address, read with scalar loads (through the constant address space): the
// descriptors of the batched passes' work items, so that an item's prologue does not wait
// on a chain of vector loads.
template <typename T> __device__ __forceinline__ T uniform_load(const T *g)
{
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    typedef const __attribute__((address_space(4))) Words<sizeof(T) / 4> *const_ptr;
    return __builtin_bit_cast(T, *(const_ptr)g);
}

// Workgroups of the batched passes hold at most 512 threads, so the persistent kernels,
// which keep a run's scalars live across work items, have up to 256 VGPRs (no spills).
constexpr int kBatchMaxThreads = 512;
// Particles per thread per batch in the batched passes: the packed state of an ensemble is
// usually larger than the Infinity Cache and streams from HBM, whose longer latency wants
// more loads in flight than the plain passes (U = 2).
template <int NV> constexpr int kBatchUnroll = NV == 1 ? 4 : 2;

struct Batch {
    const BatchRun *runs;
    const BatchItem *items;
    int32_t nitems, nruns;
    double *X, *V;         // packed particle arrays
    int64_t *stepc;        // steps completed (device counter)
};

// The per-step arrays of a run with those of parity par at index 0: the pass bodies then
// index them with constants (par = 0), which keeps the copied descriptor in registers
// rather than in scratch memory.
__device__ __forceinline__ Work by_parity(Work w, int par)
{
    if (par) {
        const double *t[4] = {w.Ef[0], w.Bf[0], w.J1[0], w.J2[0]};
        w.Ef[0] = w.Ef[1];
        w.Bf[0] = w.Bf[1];
        w.J1[0] = w.J1[1];
        w.J2[0] = w.J2[1];
        w.Ef[1] = const_cast<double *>(t[0]);
        w.Bf[1] = const_cast<double *>(t[1]);
        w.J1[1] = const_cast<double *>(t[2]);
        w.J2[1] = const_cast<double *>(t[3]);
    }
    return w;
}

template <int ORDER, int NV, bool EM, int DEP>
__global__ __launch_bounds__(kBatchMaxThreads) void k_batch_pass_a(Batch b)
{
    extern __shared__ double smem[];
    __shared__ double red[kRedSize];
    __shared__ int wctr;
    const int64_t step = uniform_load(b.stepc);
    const int par = (int)(step & 1);
    for (int it = blockIdx.x; it < b.nitems; it += gridDim.x) {
        const BatchItem item = uniform_load(b.items + it);
        const BatchRun br = uniform_load(b.runs + item.run);
        const Run &r = br.r;
        const Work wk = by_parity(br.wk, par);
        pass_a_body<ORDER, NV, EM, DEP, kBatchUnroll<NV>>(r, wk, 0, step, b.X + br.poff,
                                                          b.V + br.poff, item.p0, item.p1,
                                                          item.slot == 0, smem, red, &wctr);
        lds_barrier();
    }
}

template <int ORDER, int NV, bool EM, bool PRED, int DEP>
__global__ __launch_bounds__(kBatchMaxThreads) void k_batch_pass_b(Batch b)
{
    extern __shared__ double smem[];
    __shared__ double red[kRedSize];
    __shared__ int wctr;
    const int par = (int)(uniform_load(b.stepc) & 1);
    for (int it = blockIdx.x; it < b.nitems; it += gridDim.x) {
        const BatchItem item = uniform_load(b.items + it);
        const BatchRun br = uniform_load(b.runs + item.run);
        const Run &r = br.r;
        const Work wk = by_parity(br.wk, par);
        pass_b_body<ORDER, NV, EM, PRED, DEP, kBatchUnroll<NV>>(
            r, wk, 0, b.X + br.poff, b.V + br.poff, b.X + br.poff, b.V + br.poff, item.p0,
            item.p1, item.slot == 0, item.slot, smem, red, &wctr);
        lds_barrier();
    }
}

// Advance the step counter (one thread, after both passes of a step).
__global__ void k_batch_tick(Batch b)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *b.stepc += 1;
}

// One workgroup per run: newest record and fields into the caller's arrays.
__global__ __launch_bounds__(1024) void k_batch_finish(Batch b)
{
    __shared__ double red[kRedSize];
    const int64_t step = *b.stepc;
    const BatchRun &br = b.runs[blockIdx.x];
    const Run r = uniform_copy(br.r);
    const Work wk = uniform_copy(br.wk);
    finish_body(r, wk, (int)(step & 1), step, red);
}

template <int NV>
__global__ __launch_bounds__(1024) void k_batch_init_particles(Batch b)
{
    __shared__ double red[kRedSize];
    for (int it = blockIdx.x; it < b.nitems; it += gridDim.x) {
        const BatchItem item = b.items[it];
        const BatchRun &br = b.runs[item.run];
        const Run r = uniform_copy(br.r);
        const Work wk = uniform_copy(br.wk);
        init_particles_body<NV>(r, wk, b.X + br.poff, b.V + br.poff, item.p0, item.p1, item.slot,
                                red);
        __syncthreads();
    }
}

template <int ORDER>
__global__ __launch_bounds__(1024) void k_batch_deposit_rho(Batch b)
{
    extern __shared__ double smem[];
    for (int it = blockIdx.x; it < b.nitems; it += gridDim.x) {
        const BatchItem item = b.items[it];
        const BatchRun &br = b.runs[item.run];
        const Run r = uniform_copy(br.r);
        const Work wk = uniform_copy(br.wk);
        deposit_rho_body<ORDER>(r, wk, b.X + br.poff, item.p0, item.p1, smem);
        __syncthreads();
    }
}

template <int ORDER, int NV, bool EM>
__global__ __launch_bounds__(1024) void k_batch_predeposit(Batch b)
{
    extern __shared__ double smem[];
    for (int it = blockIdx.x; it < b.nitems; it += gridDim.x) {
        const BatchItem item = b.items[it];
        const BatchRun &br = b.runs[item.run];
        const Run r = uniform_copy(br.r);
        const Work wk = uniform_copy(br.wk);
        predeposit_body<ORDER, NV, EM>(r, wk, b.X + br.poff, b.V + br.poff, item.p0, item.p1, smem);
        __syncthreads();
    }
}

// One workgroup per run.
__global__ __launch_bounds__(1024) void k_batch_fx_setup(Batch b)
{
    __shared__ double red[kRedSize];
    const BatchRun &br = b.runs[blockIdx.x];
    const Run r = uniform_copy(br.r);
    const Work wk = uniform_copy(br.wk);
    fx_setup_body(r, wk, red);
}

__global__ __launch_bounds__(1024) void k_batch_gauss(Batch b)
{
    extern __shared__ double smem[];
    const BatchRun &br = b.runs[blockIdx.x];
    const Run r = uniform_copy(br.r);
    const Work wk = uniform_copy(br.wk);
    gauss_body(r, wk, smem);
}

__global__ __launch_bounds__(1024) void k_batch_cn_init(Batch b)
{
    const BatchRun &br = b.runs[blockIdx.x];
    const Run r = uniform_copy(br.r);
    const Work wk = uniform_copy(br.wk);
    cn_init_body(r, wk);
}

__global__ __launch_bounds__(1024) void k_batch_init_finish(Batch b)
{
    __shared__ double red[kRedSize];
    const BatchRun &br = b.runs[blockIdx.x];
    const Run r = uniform_copy(br.r);
    const Work wk = uniform_copy(br.wk);
    init_finish_body(r, wk, red);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *b.stepc = 0;
}

}  // namespace pic
