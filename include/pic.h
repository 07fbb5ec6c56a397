/*
 * pic.h -- C ABI of the MI355X (gfx950) PIC-MCC thermionic-diode library.
 *
 * The library advances the 1D3V electrostatic particle-in-cell / Monte Carlo
 * collision model of a thermionically emitting helium cathode-anode diode of
 * Zhang, Zhou and Zhao (electron transpiration cooling): every step gathers
 * the field, pushes particles (leapfrog), absorbs them at the electrodes,
 * applies null-collision MCC against a uniform helium background, injects
 * thermionic electrons and replenished pairs, deposits charge and solves the
 * 1D Poisson problem ("Model": numerical setup; "Emission and collisions").
 * Diagnostics follow "Benchmark cases" and "Boundary energy diagnostics",
 * eqs. 1-10.
 *
 * Conventions (all entry points):
 *  - SI units; temperatures in eV.
 *  - Species: 0 plasma electrons, 1 emitted electrons, 2 He+ ions.
 *    Walls: 0 cathode (z = 0, phi = 0), 1 anode (z = L, phi = V).
 *    Channels: 0 e-He elastic, 1 excitation, 2 ionisation, 3 He+-He charge
 *    exchange, 4 He+-He elastic.
 *  - Ownership: the caller owns the device workspace and the HIP stream; the
 *    library owns only the host-side handle and never frees caller memory.
 *  - Errors: every call returns 0 or a negative PIC_E* code; no exception
 *    crosses the ABI.  pic_last_error() gives a message.  Device-side
 *    conditions (capacity, null-collision bound, queue overflow) are sticky
 *    bits reported by the next synchronising call.
 *  - Asynchrony: pic_step only enqueues work on the bound stream.  Calls that
 *    return host data synchronise that stream first.
 *  - Device pointers are hipMalloc-compatible (e.g. a torch uint8 CUDA tensor);
 *    host pointers are ordinary host memory.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_OK 0
#define PIC_EINVAL (-1)     /* bad argument or configuration */
#define PIC_ENOSPACE (-2)   /* workspace too small or particle capacity exceeded */
#define PIC_EHIP (-3)       /* HIP runtime error */
#define PIC_ENULLCOLL (-4)  /* a candidate's collision frequency exceeded nu_max */
#define PIC_ENAN (-5)       /* non-finite particle state */
#define PIC_ERANGE (-6)     /* a queue or histogram bound was exceeded: the ionisation queue
                               (4096 events per diode and step), or a node's deposit reaching
                               2^53 (2^21 particles of one species on one node), beyond which
                               FP64 densities are no longer exact */

#define PIC_MAX_DIODES 256

/* One diode.  Filled by the caller; read by pic_workspace_size / pic_init. */
typedef struct pic_config {
    double L;             /* gap length (m) */
    int32_t N;            /* cells; nodes 0..N; N >= 2 */
    int32_t flags;        /* reserved, must be 0 */
    double V;             /* anode potential (V) */
    double n0;            /* initial plasma density (m^-3) */
    double Te0, Ti0;      /* initial electron / ion temperature (eV) */
    int64_t n_load;       /* macro-particles per species (electrons, ions) at load */
    double gamma_emit;    /* imposed emitted-electron flux (m^-2 s^-1) */
    double Tc;            /* emission temperature (eV) */
    double ng;            /* neutral density (m^-3) */
    double Tne, Tni;      /* neutral target temperature, e / ion collisions (eV) */
    double dt;            /* time step (s) */
    double sig_el;        /* e-He elastic cross section (m^2), energy independent */
    double sig_x0;        /* excitation scale (m^2): sig_x0 ln(x)/x, x = eps/19.82 eV */
    double lotz_a;        /* ionisation: Lotz a (m^2 eV^2), q = 2, threshold 24.59 eV */
    double sig_cx;        /* He+-He charge exchange (m^2), energy independent */
    double sig_iel;       /* He+-He elastic (m^2), energy independent */
    uint32_t channels;    /* bit c enables channel c */
    int32_t replenish;    /* 1: re-inject one e-ion pair per ion lost ("Model") */
    uint32_t seed;        /* Philox key word 1 = seed ^ diode */
    uint32_t diode;       /* index used in the key */
    int32_t tally_period; /* D: tallies snapshot every D steps (>= 1) */
    int32_t sort_period;  /* K: cell re-sort every K steps (0: library default) */
    double capacity_factor; /* slots per species = factor * n_load (0: 1.6) */
} pic_config;

/* Cumulative raw tallies of one diode since pic_init. */
typedef struct pic_tally {
    int64_t step;                 /* completed steps */
    int64_t n_live[3];            /* live particles per species */
    int64_t abs_count[3][2];      /* particles absorbed per species and wall */
    double abs_energy[3][2];      /* sum over them of 1/2 m |v|^2 (J per macro-particle) */
    int64_t n_emit, n_repl, n_iz; /* emitted, replenished pairs, ionisation events */
    int64_t cand[2];              /* null-collision candidates (electrons, ions) */
    int64_t coll[5];              /* real collisions per channel */
    uint32_t next_id;             /* next particle id */
    uint32_t err_bits;            /* sticky device error bits */
    int64_t rare_spill;           /* collision candidates and absorbed particles that the particle
                                     kernel's per-wave queues could not hold and handed to the
                                     sources kernel (a work-list counter, not physics) */
    int64_t resorts;              /* cell re-sorts of the particle stores so far */
    int64_t resorts_ions_kept;    /* of them, those that left the ions where they were (they move a
                                     fraction of a cell per re-sort period; a schedule counter, not
                                     physics) */
} pic_tally;

/* Boundary diagnostics over a window ("Benchmark cases", eqs. 1-10). */
typedef struct pic_diag {
    int64_t step_begin, step_end; /* window [begin, end) in steps */
    double gamma_emit;            /* imposed Gamma_emit */
    double gamma_emit_meas;       /* injected macro-electrons * w0 / window */
    double gamma_ref;             /* emitted electrons returning to the cathode */
    double gamma_net;             /* Gamma_emit - Gamma_ref */
    double gamma_anode;           /* emitted electrons collected at the anode */
    double backflow_pct;          /* 100 Gamma_ref / Gamma_emit */
    double eta_net, eta_anode;    /* Gamma_net / Gamma_emit, Gamma_anode / Gamma_emit */
    double gamma_abs[3][2];       /* particle flux per species and wall (m^-2 s^-1) */
    double q_abs[3][2];           /* kinetic energy flux per species and wall (W m^-2) */
    double wf_eff;                /* eq. 2 (eV) */
    double q_emit_theory;         /* eq. 1 */
    double q_ion_cath_recomb;     /* eq. 3 */
    double q_cool1, q_cool2;      /* eqs. 4, 5 */
    double q_ion_anode_recomb;    /* eq. 7 */
    double q_anode1, q_anode2;    /* eqs. 6, 8 */
    double phi_vc_eff;            /* eq. 10 (V); NaN if Gamma_net <= 0 */
    double n_live[3];             /* live particles at the window end */
} pic_diag;

/* Quantities derived from a configuration on the host (no GPU needed). */
typedef struct pic_derived {
    double dz, invdz, w0;         /* cell, 1/cell, macro-weight n0 L / n_load (m^-2) */
    double numax[2];              /* null-collision bound, electrons / ions (s^-1) */
    double lam[2];                /* numax * dt */
    double emit_per_step;         /* Gamma_emit dt / w0 */
    int64_t capacity[3];          /* particle slots per species */
} pic_derived;

/* Steady-state verdict of one diode (see pic_steady_state). */
typedef struct pic_steady {
    int32_t steady;            /* 1 if the criterion was met */
    int32_t blocks;            /* complete blocks examined */
    int64_t block_steps;       /* steps per block */
    int64_t steady_step;       /* end step of the first steady block, -1 if none */
    double backflow_pct;       /* mean backflow ratio of the blocks after it (NaN if none) */
    int32_t blocks_averaged;   /* how many blocks entered that mean (<= 4) */
    int32_t pad;
    double last_backflow_pct;  /* backflow ratio of the last complete block */
} pic_steady;

typedef struct pic_handle pic_handle;

/* Derived parameters of one configuration ("Model": w0 = n0 dz / N_ppc;
 * null-collision bound per species).  Host only.  PIC_EINVAL on a bad config. */
int pic_derive(const pic_config *cfg, pic_derived *out);

/* Device workspace bytes for n_diodes diodes (1 <= n_diodes <= PIC_MAX_DIODES). */
int pic_workspace_size(const pic_config *cfgs, int n_diodes, size_t *bytes);

/* Create a handle over a caller-owned device workspace of at least
 * pic_workspace_size bytes (256-byte aligned), bound to hip_stream (a
 * hipStream_t; NULL = default stream).  Enqueues the initial load (uniform
 * positions, Maxwellian velocities; "Model"), the first deposit and the first
 * field solve.  Asynchronous. */
int pic_init(const pic_config *cfgs, int n_diodes, void *dev_workspace, size_t bytes,
             void *hip_stream, pic_handle **out);

/* Warm start: as pic_init, but the particles follow given densities instead
 * of the uniform n0 (the loaded state of "Model" with n(z) in place of n0).
 * dev_dens is a device array [n_diodes][2][Nmax] of doubles (m^-3): row 0 the
 * electron density, row 1 the ion density at the N cell centres of each diode
 * (Nmax = the largest N; shorter rows are padded and ignored).  Cell c of a
 * species receives floor(x) particles plus one with probability frac(x),
 * x = n_c dz / w0 (w0 from the configuration as in pic_init), drawn from
 * Philox keyed by the cell; positions are uniform in the cell, velocities
 * Maxwellian at Te0 / Ti0, electrons join the plasma population, ids run over
 * the electron cells then the ion cells.  The array is read before return
 * (the call synchronises the stream).  PIC_ENAN for a negative or non-finite
 * density, PIC_ENOSPACE when a species exceeds its capacity
 * (capacity_factor x n_load). */
int pic_init_from_profiles(const pic_config *cfgs, int n_diodes, void *dev_workspace, size_t bytes,
                           void *hip_stream, const double *dev_dens, pic_handle **out);

/* Warm start from a late-time state: as pic_init_from_profiles, with the
 * velocities drawn from per-cell summaries of a late-time velocity
 * distribution instead of the load Maxwellians (a reading: the paper starts
 * every run from the uniform Maxwellian load).  dev_state is a device array
 * [n_diodes][PIC_STATE_ROWS][Nmax] of doubles on the N cell centres:
 *   row 0 n_e, row 1 n_i (m^-3; as the two rows of pic_init_from_profiles),
 *   row 2 the potential phi (V),
 *   rows 3..11 electron v_z quantiles, rows 12..20 electron |v_perp|
 *   quantiles, rows 21..29 ion v_z quantiles, rows 30..38 ion |v_perp|
 *   quantiles (m/s), at the levels 0, 0.02, 0.1, 0.25, 0.5, 0.75, 0.9, 0.98, 1.
 * Counts, ids, positions and free flights are those of
 * pic_init_from_profiles for the same densities.  Each nine-vector is sorted
 * first; v_z and |v_perp| are drawn from the piecewise-linear inverse of the
 * cell's quantile function with two uniform draws, the azimuth of (v_x, v_y)
 * uniformly with a third (Philox keyed by the particle id, event LOAD, counter
 * word 2 = 0, 0, 2).  A particle whose kinetic energy exceeds the
 * null-collision bound's energy cap, e (|V| + 40 Te0 + 40 Tc) (electrons) or
 * e (|V| + 40 Ti0) (ions), is scaled down to it.  Row 2 (phi) is checked
 * for being finite and otherwise not read.
 * Reads the array before return.  PIC_ENAN for a negative density or a
 * non-finite entry, PIC_ENOSPACE as for pic_init_from_profiles. */
#define PIC_STATE_ROWS 39
int pic_init_from_state(const pic_config *cfgs, int n_diodes, void *dev_workspace, size_t bytes,
                        void *hip_stream, const double *dev_state, pic_handle **out);

/* Advance every diode nsteps steps.  Asynchronous on the bound stream. */
int pic_step(pic_handle *h, int64_t nsteps);

/* Synchronise the bound stream; return the first sticky device error, if any. */
int pic_sync(pic_handle *h);

/* Raw cumulative tallies of one diode.  Synchronises. */
int pic_get_tally(pic_handle *h, int diode, pic_tally *out);

/* The tallies of one diode as they stood at the end of step `step` (a
 * multiple of tally_period, taken from the snapshot ring, so at most 1024
 * tally periods back; step 0 gives zeros).  next_id is 0; err_bits is the
 * current value.  PIC_EINVAL for a step that is not a tally step or not yet
 * reached, PIC_ERANGE once it has left the ring.  Synchronises. */
int pic_get_snapshot(pic_handle *h, int diode, int64_t step, pic_tally *out);

/* Boundary diagnostics of one diode over the last window_steps steps
 * (a multiple of tally_period and at most tally_period * 1024 steps back), or
 * since the initial load when window_steps == 0.  Synchronises. */
int pic_diagnostics(pic_handle *h, int diode, int64_t window_steps, pic_diag *out);

/* Node profiles of one diode (N+1 doubles each, any pointer may be NULL):
 * phi (V), electron density (both populations) and ion density (m^-3) from
 * the last deposit, or time averages since pic_avg_reset when time_avg != 0.
 * Boundary nodes carry half-cell volumes.  Synchronises. */
int pic_get_fields(pic_handle *h, int diode, double *phi, double *n_e, double *n_i, int time_avg);

/* Start (on != 0) or stop time averaging of phi and densities. */
int pic_avg_reset(pic_handle *h, int on);

/* The same for one diode (diode = -1: all): clears its sums and sets its
 * averaging flag, leaving the other diodes' averages untouched.  Lets each
 * diode of a batch average over its own late-time window.  Synchronises. */
int pic_avg_control(pic_handle *h, int diode, int on);

/* Raw per-species fixed-point deposit of the last step (N+1 int64; a particle
 * deposits 2^32 in total).  Synchronises. */
int pic_get_hist(pic_handle *h, int diode, int species, int64_t *out);

/* Field at the nodes used by the next push (N+1 doubles).  Synchronises. */
int pic_get_efield(pic_handle *h, int diode, double *out);

/* Phase-space histogram of one species of one diode (the kinetic diagnostics
 * of "Phase-space and velocity-distribution characteristics": (z, v_z)
 * phase space, and by summing rows, the gap-integrated and the regional axial
 * velocity distributions).  Adds to dev_out (device memory, caller-owned and
 * caller-cleared, nz rows of nv + 2 uint64, row-major) the number of live
 * particles in each bin as they stand after all work enqueued so far:
 *   row    iz = min(nz - 1, floor(z * (nz / L)))
 *   column with x = (v_z - vmin) * (nv / (vmax - vmin)), both factors in FP64:
 *          0 if x < 0, 1 + floor(x) if 0 <= x < nv, nv + 1 if x >= nv.
 * v_z is the stored leapfrog velocity (m/s, half a step behind z).  Species
 * 0 plasma electrons, 1 emitted electrons, 2 ions.  Requires nz >= 1,
 * nv >= 1, nz * (nv + 2) <= PIC_PHASE_MAX_BINS, finite vmin < vmax and
 * dev_out in device memory of the handle's GPU (else PIC_EINVAL).  Enqueued on the handle's stream; does not synchronise.
 * Calls that add into one buffer accumulate (a late-time average is a sum of
 * samples). */
#define PIC_PHASE_MAX_BINS 32768
int pic_phase_space(pic_handle *h, int diode, int species, int nz, int nv, double vmin, double vmax,
                    uint64_t *dev_out);

/* Live particles of one species, sorted by id, into host arrays of capacity
 * cap; *n_out receives the count (PIC_ENOSPACE if cap is too small).  Any
 * array may be NULL.  tc is the step at which the particle is next a
 * null-collision candidate.  Synchronises. */
int pic_get_particles(pic_handle *h, int diode, int species, int64_t cap, int64_t *n_out,
                      double *z, float *vx, float *vy, float *vz, uint32_t *id, uint32_t *tc);

/* Replace one species of one diode by n host particles (cell order need not be
 * kept: the next step re-sorts).  Every z must lie in (0, L) (PIC_EINVAL
 * otherwise) and every velocity component be finite (PIC_ENAN otherwise);
 * nothing is changed on an error.  tc is the step at which the particle is
 * next a null-collision candidate.  Synchronises. */
int pic_set_particles(pic_handle *h, int diode, int species, int64_t n, const double *z,
                      const float *vx, const float *vy, const float *vz, const uint32_t *id,
                      const uint32_t *tc);

/* Set the step counter and next particle id of one diode. */
int pic_set_counters(pic_handle *h, int diode, int64_t step, uint32_t next_id);

/* Re-deposit the current particles and re-solve the field without stepping. */
int pic_refield(pic_handle *h);

/* Per-kernel timing: run nsteps steps on the current schedule -- with graph
 * replay, each run up to the next re-sort boundary is one replayed graph, as
 * in pic_step -- with HIP events around launches of the particle kernel on
 * the bound stream (with graph replay: the particle kernels of up to 8 steps
 * spread evenly over each replayed run, at most 4096 in all; on the plain
 * stream, where each pair of timestamps stalls the launches around it, at
 * most 32: every launch when nsteps <= w, else one in s = ceil(nsteps / w)
 * rounded up to an odd number, w = min(32, max(4, nsteps / 16))) and return
 * their mean duration and the time from the first enqueued step to the end
 * of the last (ms).
 * Events are created on first use and kept by the handle.  Synchronises at
 * the end only. */
int pic_step_timed(pic_handle *h, int64_t nsteps, double *particle_kernel_ms, double *total_ms);

/* Launch schedule of the hot loop: particles per thread in the particle and
 * sort kernels (1, 2, 4 or 8; 0 keeps), persistent grid size (0: default),
 * re-sort period in steps (0 keeps) and whether full re-sort periods are
 * replayed from a captured HIP graph (-1 keeps).  Results do not depend on
 * these choices.  Synchronises. */
int pic_set_tuning(pic_handle *h, int ppt, int grid, int sort_period, int use_graph);
int pic_get_tuning(pic_handle *h, int *ppt, int *grid, int *sort_period, int *use_graph);

/* Choose the launch schedule by timing candidates on the handle's own
 * diodes: every combination of particles per thread {1, 2, 4}, re-sort period
 * {16, 32, 64, 128} and grid {2048, 3072, 4096, 6144, 8192, 12288, 16384, and
 * the grid that gives each block eight chunks of the current particles (a
 * multiple of 8 in 256..65536)}; the best four timed twice
 * more; then graph replay on or off for the best one.  Each candidate runs
 * whole re-sort periods of at least trial_steps real steps, so the diodes
 * advance.  Leaves the best schedule set and returns it with its time per
 * step.  Synchronises. */
int pic_autotune(pic_handle *h, int64_t trial_steps, int *ppt, int *grid, int *sort_period, int *use_graph,
                 double *ms_per_step);

/* Late-time steady state ("Benchmark cases": fluxes are averaged over late
 * intervals in which they fluctuate around stable means; the paper leaves the
 * interval choice open).  Tallies are grouped in blocks of block_tallies
 * snapshots; block b is steady when its backflow ratio differs from those of
 * blocks b-1 and b-2 by less than tol_pp percentage points and its live
 * particle count from that of block b-1 by less than the fraction tol_rel.
 * The steady backflow ratio is the mean over the up to four following blocks.
 * Uses the snapshot ring, so it sees at most 1024 tally periods.  Synchronises. */
int pic_steady_state(pic_handle *h, int diode, int block_tallies, double tol_pp, double tol_rel,
                     pic_steady *out);

/* The same criterion on host series of per-block backflow ratios (percent) and
 * live counts: *steady_block is the first steady block (-1 if none),
 * *br_steady the mean of up to four following blocks, *n_mean how many.
 * Host only. */
int pic_steady_from_series(const double *br, const double *n_live, int nblocks, double tol_pp, double tol_rel,
                           int *steady_block, double *br_steady, int *n_mean);

/* Message of the last failing call on this thread. */
const char *pic_last_error(void);

/* Checkpoint / restart.  pic_save writes a host image of every diode's
 * state at the current step boundary: configuration, state block, tallies,
 * snapshot ring, node arrays (deposits, their sums, phi, E) and the particle
 * slots of the current buffer.  pic_checkpoint_size gives the bytes it needs
 * (it grows with the live counts).  pic_load restores such an image into a
 * handle created with the same configurations (physics fields compared;
 * PIC_EINVAL otherwise, PIC_ENOSPACE if the particles exceed its capacity);
 * the next step re-sorts.  A restored run continues as the saved one would
 * have: particles, deposits and integer tallies bit for bit (the FP64
 * absorbed-energy sums up to the order of their additions).  All three
 * synchronise; the buffer is the caller's. */
int pic_checkpoint_size(pic_handle *h, size_t *bytes);
int pic_save(pic_handle *h, void *host_buf, size_t bytes, size_t *written);
int pic_load(pic_handle *h, const void *host_buf, size_t bytes);

/* Release the handle (not the caller's workspace or stream). */
void pic_destroy(pic_handle *h);

#ifdef __cplusplus
}
#endif
#endif
