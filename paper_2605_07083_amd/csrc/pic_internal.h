// pic_internal.h -- device-resident data layout of the gfx950 PIC-MCC library.
//
// Every diode of a handle owns, inside the caller's workspace:
//   * two particle buffers per species (ping-pong for the cell re-sort):
//     arrays z f64, vz f32, tc u32 and an array of 16-byte {vx, vy, id}
//     records;
//   * three fixed-point deposit histograms (int64, N+1 nodes) plus copies of
//     the last step's, phi and E (f64, N+1), time-average accumulators;
//   * sort scratch (one int32 per 32-cell bin and species), the ionisation queue,
//     the mutable state block, cumulative tallies and a ring of snapshots.
// The hot loop streams z (r/w), vz (r/w) and tc (r) only; vx, vy and id are
// touched for null-collision candidates and absorbed particles, which the hot
// loop lists per species (one u32 per slot of capacity) for the sources
// kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int NSP = 3;
constexpr int SP_P = 0, SP_E = 1, SP_I = 2;
constexpr int NCH = 5;
constexpr int CH_EEL = 0, CH_EXC = 1, CH_IZ = 2, CH_CX = 3, CH_IEL = 4;
constexpr uint32_t EV_COLL = 1, EV_LOAD = 2, EV_EMIT = 3, EV_BIRTH = 4, EV_PROFILE = 5;
constexpr uint32_t LOAD_STEP = 0xFFFFFFFFu;
constexpr uint32_t NEVER = 0xFFFFFFFFu;
constexpr int RING = 1024;           // tally snapshots kept per diode
constexpr int IZQ_CAP = 4096;        // ionisation events per diode per step
constexpr int MAX_DIODES = 256;
constexpr int PHASE_MAX_BINS = 32768;   // LDS counts of the phase-space histogram (128 KB)

// sticky device error bits
constexpr uint32_t ERR_CAPACITY = 1u;
constexpr uint32_t ERR_NULLCOLL = 2u;
constexpr uint32_t ERR_NAN = 4u;
constexpr uint32_t ERR_IZQ = 8u;
constexpr uint32_t ERR_RANGE = 16u;   // a node's deposit reached 2^53 (2^21 particles of one species)
constexpr unsigned long long DEPOSIT_LIMIT = 1ull << 53;

// physical constants (CODATA 2018)
constexpr double Q_E = 1.602176634e-19;
// rows of a warm-start state per diode: n_e, n_i, phi, then per species
// (electrons, ions) nine quantiles of v_z and nine of |v_perp|
constexpr int STATE_ROWS = 39;
constexpr double K_B = 1.380649e-23;
constexpr double EPS0 = 8.8541878128e-12;
constexpr double MASS_E = 9.1093837015e-31;
constexpr double MASS_HE = 6.6464731e-27;
constexpr double E_EXC = 19.82;
constexpr double E_ION = 24.59;

// Fields touched only by collision candidates, absorbed particles, births
// and the re-sort, kept together so that such a particle costs one 16-byte
// access instead of three scattered 4-byte ones.
struct ColdRec {
    float vx, vy;
    uint32_t id;
    uint32_t pad;
};

struct SpeciesBuf {
    double *z;          // streamed every step
    float *vz;          // streamed every step
    uint32_t *tc;       // streamed every step (read)
    ColdRec *cold;      // v_x, v_y, id
};

// Nodes per tile of the large-grid field kernel (one aggregate and flag each).
constexpr int FIELD_BIG_TILE = 512;

// Mutable per-diode state (device).
struct DiodeState {
    int32_t n[NSP];        // slots in use in the current buffer (live + holes)
    int32_t n_new[NSP];    // live count found by the re-sort
    int32_t parity;        // which buffer is current
    uint32_t next_id;
    uint32_t step;
    int32_t iz_count;      // ionisation events queued this step
    int32_t ion_lost;      // ions absorbed this step
    uint32_t err;
    int32_t avg_on;
    int32_t avg_steps;
    int32_t rare_n[NSP];   // rare items (candidates, absorbed) listed this step
    int32_t arrive;        // field step: blocks that have read this step's counters
    uint32_t spill_flag;   // field step: step + 1 once the spilled rare items are done
    uint32_t field_epoch;  // large-grid field step: launches so far (tile aggregate flags are epoch + 1)
    // Species s lives in buffer parity ^ flip[s]: a re-sort that keeps a
    // species where it is (keep[s], decided by the re-sort's scan) flips the
    // diode's parity but not the species' buffer, so it toggles flip[s].
    int32_t flip[NSP];
    int32_t keep[NSP];
    uint32_t resorts;      // re-sorts so far
    uint32_t rec_flag;     // field step: step + 1 once the record block's newborns and tallies are done
    // Large-grid field step (zero on smaller grids): the stored phi and E
    // leave out phi_slope j and e_shift = -phi_slope / dz, the part of the
    // potential that needs every tile; phi_slope_sum is the slope's sum over
    // the steps of the time average.
    double phi_slope;
    double e_shift;
    double phi_slope_sum;
};

// Cumulative tallies (device); all integers are order independent.
struct DiodeTally {
    unsigned long long abs_count[NSP][2];
    double abs_energy[NSP][2];
    unsigned long long n_emit, n_repl, n_iz;
    unsigned long long cand[2];
    unsigned long long coll[NCH];
    unsigned long long rare_spill;   // rare items the particle kernel moved to the global lists
    unsigned long long resorts;      // re-sorts
    unsigned long long resorts_ions_kept;   // of them, those that left the ions in place
};

struct TallySnap {
    unsigned long long step;
    DiodeTally t;
};

struct IzEvent {
    double z;
    uint32_t parent;
    float ve[3];   // secondary electron
    float vi[3];   // new ion
    uint32_t pad;
};

// Tallies of one block's rare work (collision candidates, absorbed
// particles), accumulated in LDS and flushed once: candidate and channel
// counts per electron/ion class, absorbed counts and energies per
// (species, wall), ions lost.
struct RareTally {
    unsigned int cand[2];
    unsigned int coll[NCH];
    unsigned int abs_count[NSP][2];
    int ion_lost;
    double abs_energy[NSP][2];
};

// The particle kernel's blocks add their tallies into TALLY_COPIES copies,
// 256 bytes apart (block b into copy b mod TALLY_COPIES): device-scope
// atomics on one address from thousands of blocks would queue on one memory
// channel.  The sources kernel folds the copies into the tallies each step.
constexpr int TALLY_COPIES = 64;
struct alignas(256) TallyCopy {
    RareTally t;
};

// Per-tile aggregates of the tiled field solve: A = sum of rho over the tile,
// B (128-bit, lo/hi) = sum over its interior nodes of the in-tile inclusive
// prefix of rho, n = its interior node count.
struct FieldAgg {
    long long A;
    unsigned long long B_lo;
    long long B_hi;
    int32_t n;
    int32_t pad;
};

// Read-only parameters and buffer pointers of one diode (device copy).
struct Diode {
    double L, dz, invdz, V, dt, w0;
    double alpha;          // e w0 dz / (2^32 eps0): node charge -> Poisson rhs
    int32_t N;
    int32_t cap[NSP];
    double qmdt[NSP];      // (q/m) dt
    double mass[NSP];
    double numax[2], lam[2];
    float numax_f[2];
    float sig_n[2];        // neutral thermal speed per axis (e, ion collisions)
    float half_mu_over_e[2];
    float mfrac_m[2];      // m / (m + M)
    float mfrac_M[2];      // M / (m + M)
    float two_e_over_mu[2];
    float ng, sig_el, sig_x0, lotz_a2, sig_cx, sig_iel;
    double emit_x;         // Gamma dt / w0
    double sig_c, sig_e0, sig_i0;
    double load_cap_ev[2]; // state load: kinetic energy limit (eV), electrons / ions
    uint32_t kseed, channels;
    int32_t replenish, tally_period;
    SpeciesBuf buf[2][NSP];
    unsigned long long *H[NSP];
    long long *Hlast[NSP];
    long long *Hsum[NSP];
    double *phi, *E, *phi_sum;
    int32_t *cell_cnt[NSP];     // per-bin counts / offsets of the re-sort
    IzEvent *izq;
    DiodeState *st;
    DiodeTally *tally;
    TallySnap *ring;
    FieldAgg *agg;         // the large-grid field step's tile aggregates
    uint32_t *agg_flag;    // and their flags (field_epoch + 1 once published)
    uint32_t *rare[NSP];   // the step's rare items per species: slot | kind << 30
    TallyCopy *tacc;       // TALLY_COPIES accumulators of the particle kernel's tallies
};

}  // namespace pic
