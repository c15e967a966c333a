// Constants and plain data shared by the device code and the host runtime of the PIC
// library (no HIP: the host-only runtime in pic_host.cpp also builds with a plain C++
// compiler).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace pic {

constexpr int kMaxGrid = 8192;   // upper bound on particle-pass workgroups
// Per-workgroup scalars: KE, fallbacks, max|G-1|, nonfinite (every pass B), and at
// initialisation also sum w, max w and max w |v| (slots 4-6, for the fixed-point scales).
constexpr int kNS = 8;
constexpr int kGhost = 4;        // ghost nodes on each side of an LDS field or current tile
constexpr int kVBins = 2;        // rebin key: cell x sign of v_x

// Upper bound on the replicas of the currents: a default launch (256 workgroups) uses 8,
// and a prologue keeps the replicas of two currents in flight at once.
constexpr int kMaxRep = 8;

// Run::scheme of the standard explicit scheme (section 5's comparison scheme) and of
// EMEC(PSATD) (section 4.2).
constexpr int kStandard = 3;
constexpr int kPsatd = 4;
constexpr int kLeapfrog = 5;     // EMEC(LF) (section 4.1)

// Convolution rows of the electromagnetic field updates (Work::prow), [kPsatdRows][ng]:
// for the predictor update (over dt/2) and the full update (over dt), the rows that map
// E (node), -B or B (half node) and j (node) of one transverse pair to the new E and B,
// then the rows of the E that v-dagger gathers (EMEC(PSATD): the time average over the
// step; EMEC(LI): the mean of E^n and E^{n+1}).
enum PsatdRow {
    kRowC1 = 0, kRowEB1, kRowEJ1, kRowBE1, kRowBJ1,     // tau1 = dt/2
    kRowC2, kRowEB2, kRowEJ2, kRowBE2, kRowBJ2,         // tau2 = dt
    kRowAE, kRowAB, kRowAJ,                             // time average over dt
    kPsatdRows
};

// Offset (in doubles) of the coefficient tiles in the LDS of the passes, kept even so that
// tent coefficients can be read as pairs.
constexpr int coef_offset(int doubles) { return (doubles + 1) & ~1; }

// Per-step record, laid out exactly like pic_diag.
struct DevRecord {
    int64_t step;
    double time, kinetic, field_e, field_b, total, rel_energy_err, max_gamma_dev;
    int64_t fallbacks, fallbacks_total;
    int32_t nonfinite, pad;
};

struct DevState {
    int64_t recorded;      // newest step whose record is written
    double te0;            // total energy of step 0
    int64_t fb_total;
    double we, wb;         // field energies of the newest fields (written by pass B)
    int32_t nonfinite_sticky;
    int32_t flag_a;        // set by a pass A whose deposit met a value it cannot hold
                           // (deterministic mode); taken into the next record
    // Fixed-point scales 2^S and 2^-S of the LDS deposit tiles (Depo<., ., 0>), chosen at
    // initialisation from the particles (k_fx_setup): [0] currents, [1] charge density.
    double fx_scale[2], fx_inv[2];
};

// Scalars of a run, passed by value to every kernel.
struct Run {
    int64_t np;
    int64_t vstride;       // distance between velocity components in V (N_p, or the
                           // packed total in the batched form)
    int32_t ng, nv;
    int32_t nblocks;       // workgroups of the particle passes
    int32_t rec_cap;
    int64_t chunk;         // particles per workgroup
    int32_t scheme;        // 0 ESEC2, 1 ESEC1, 2 EMEC(LI), 3 standard (kStandard),
                           // 4 EMEC(PSATD) (kPsatd), 5 EMEC(LF) (kLeapfrog)
    int32_t tw;            // LDS tile width: ng + 2 kGhost
    int32_t nrep;          // replicas of the current accumulators (see Work::J1)
    int32_t interleave;    // 1: the particle passes deal batches round-robin (WaveBatches)
    int32_t det;           // 1: deterministic mode (static batches, ordered current sums)
    int32_t filter_rho;    // standard scheme: binomial filter on the charge density
    int32_t cc;            // exact charge conservation (ESEC2, electrostatic, tents): E_x
                           // and j on the half nodes, the centred deposit and v-dagger's
                           // gather through the pieces of each path
    int32_t em_fields;     // EMEC(LI), EMEC(PSATD): a field launch before pass B computes
                           // E^{n+1}, B^{n+1} and the gathered averages (Work::pf); 0:
                           // pass B's prologue does (EMEC(LF), the batched form)
    double L, h, inv_h, dt, hdt, c2;
    double xshift;         // grid offset of E_x and j in cells: 0.5 with cc (half nodes), else 0
    double qs;             // 1/h: deposit factor (times w_p)
    double wu;             // uniform weight L / N_p
    double fx_lim;         // contributions with |c| 2^S >= fx_lim leave the fixed-point tile
                           // (each tile entry then stays below 2^62: fx_lim <= 2^62 / chunk)
    double bext[3];
    const double *w;       // [N_p] weights or nullptr (uniform)
};

// Workspace arrays (device pointers).  Index [k] below is the step parity.
struct Work {
    double *E, *B;         // caller fields: E[3][ng], B[2][ng] (B null for ES)
    double *Ef[2];         // [3][ng] E^n (Ef[n & 1])
    double *Bf[2];         // [2][ng] B^n
    // Currents are accumulated with device-scope atomics from every workgroup.  To keep
    // the chain of atomics on each address short, they go to nrep replicas [nrep][3][ng]
    // (workgroup b adds into replica b mod nrep); readers sum the replicas in order.
    double *J1[2];         // [nrep][3][ng] predictor current j^{n,*} (J1[n & 1])
    double *J2[2];         // [nrep][3][ng] centred current j^{*,n+1/2} (J2[n & 1])
    double *cninv;         // [ng] first row of the Crank-Nicolson inverse
    // EM schemes (else null): the field-update rows, the predictor fields E*[3][ng] |
    // B*[2][ng] of the current step (EMEC(PSATD)), and the E [3][ng] | B^{n+1/2} [2][ng]
    // that pass B gathers
    double *prow, *ps, *pf;
    double *grid_save;     // [6][ng] or null: pass B's lead copies E^n, j^{n,*},
                           // j^{*,n+1/2} (replicas summed) and the fields it built from
                           // them, E*, E-bar, E^{n+1}, here (adjoint recompute)
    double *spart;         // [nblocks][kNS] pass-B scalars of the newest state
    double *part;          // deterministic mode: [nblocks][3][ng] per-workgroup deposits,
                           // summed in workgroup order by k_reduce_partials
    DevState *st;
    DevRecord *rec;        // [rec_cap] ring
    // counting-sort rebin (only when enabled)
    double *x2, *v2;       // [N_p], [nv][N_p] sorted copy of the state
    int64_t *id2;          // [N_p] (ids tracked)
    double *wcur, *w2;     // [N_p] permuted weights (non-uniform weights)
    int64_t *hist;         // [nbins][nblocks] counts, then offsets
    int64_t *segsum;       // [nseg] per-segment sums of hist
};

}  // namespace pic
