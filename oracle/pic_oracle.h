/*
 * pic_oracle.h -- plain, slow FP64 CPU oracle of the 1D3V electrostatic
 * PIC-MCC thermionic diode (Zhang, Zhou, Zhao, "Full-gap kinetic limitation of
 * thermionic-electron transport for electron transpiration cooling").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no source with the HIP library.
 *
 * Units: SI, temperatures in eV.  Species 0 = plasma electrons, 1 = emitted
 * electrons, 2 = He+ ions.  Wall 0 = cathode (z = 0), wall 1 = anode (z = L).
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OSP_P = 0, OSP_E = 1, OSP_I = 2, ONSP = 3 };
enum { OCH_EEL = 0, OCH_EXC = 1, OCH_IZ = 2, OCH_CX = 3, OCH_IEL = 4, ONCH = 5 };

typedef struct {
    double L;            /* gap length (m) */
    int32_t N;           /* cells; nodes 0..N */
    int32_t periodic;    /* 1: periodic test mode (no walls, sources, collisions) */
    double V;            /* anode potential (V); cathode is 0 V */
    double n0;           /* initial plasma density (m^-3) */
    double Te0, Ti0;     /* initial electron / ion temperature (eV) */
    int64_t n_load;      /* macro-particles per species at load */
    double gamma_emit;   /* imposed emitted-electron flux (m^-2 s^-1) */
    double Tc;           /* emission temperature (eV) */
    double ng;           /* neutral density (m^-3) */
    double Tne, Tni;     /* neutral target temperature for e / ion collisions (eV) */
    double dt;           /* time step (s) */
    double sig_el;       /* e-He elastic cross section (m^2), constant */
    double sig_x0;       /* excitation scale (m^2) */
    double lotz_a;       /* Lotz ionisation constant (m^2 eV^2) */
    double sig_cx;       /* He+-He charge exchange (m^2), constant */
    double sig_iel;      /* He+-He elastic (m^2), constant */
    uint32_t channels;   /* bit c enables channel c (OCH_*) */
    int32_t replenish;   /* pair replenishment on/off */
    uint32_t seed;       /* Philox key word 1 is seed ^ diode */
    uint32_t diode;
} ocfg;

typedef struct {
    double dz, invdz, w0;
    double qm[ONSP];          /* charge / mass */
    double mass[ONSP];
    double numax[2];          /* electrons, ions (s^-1) */
    double lam[2];            /* numax * dt */
    double sig_n[2];          /* neutral thermal speed per axis for e / ion collisions */
} oderived;

typedef struct {
    int64_t abs_count[ONSP][2];
    double abs_energy[ONSP][2];    /* sum of 1/2 m |v|^2 (J) per macro-particle */
    int64_t n_emit, n_repl, n_iz;
    int64_t cand[2];               /* null-collision candidates, electrons / ions */
    int64_t coll[ONCH];
    int64_t nullcoll_exceed;       /* candidates with nu(g) > numax */
} otally;

typedef struct osim osim;

/* Primitives (each is pinned separately by the CPU tests). */
void o_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double o_u24(uint32_t w);
double o_u32(uint32_t w);
double o_u53(uint32_t hi, uint32_t lo);
double o_sigma(const ocfg *c, int channel, double eps_eV);
int o_derive(const ocfg *c, oderived *d);
void o_deposit(int64_t n, const double *z, int32_t N, double invdz, int64_t *H);
int o_solve(int32_t N, double dz, double V, const double *rho, double *phi);
void o_efield(int32_t N, double dz, const double *phi, double *E);

/* Whole simulation. */
osim *o_create(const ocfg *c);
void o_destroy(osim *o);
int o_load(osim *o);
/* Load from cell-centre densities n_e, n_i (N values each, m^-3); -2 on a
 * negative or non-finite density. */
int o_load_profiles(osim *o, const double *ne, const double *ni);

/* Warm start from a late-time state on the N cells: prof[r][c], rows
 *   0 n_e, 1 n_i (m^-3), 2 phi (V; carried with the state, not used by the load),
 *   3..11 electron v_z quantiles, 12..20 electron |v_perp| quantiles (m/s),
 *   21..29 ion v_z quantiles, 30..38 ion |v_perp| quantiles,
 * at the levels OQ_LEVELS.  Counts, ids, positions and free flights as in
 * o_load_profiles; velocities from the quantiles, kinetic energies capped at
 * the null-collision bound's energy cap.  -2: negative density or a
 * non-finite entry. */
#define OSTATE_ROWS 39
#define OQ 9
int o_load_state(osim *o, const double *prof);
int o_step(osim *o);
int o_refield(osim *o);
int64_t o_count(const osim *o, int sp);
int o_threads(void);
int64_t o_last_moves_count(const osim *o, int sp);
int64_t o_last_moves(const osim *o, int sp, uint32_t *id, double *z, int32_t *fate, int32_t *ch,
                     double *margin);
int64_t o_stepno(const osim *o);
uint32_t o_next_id(const osim *o);
void o_set_counters(osim *o, int64_t step, uint32_t next_id);
int o_get_particles(const osim *o, int sp, double *z, double *vx, double *vy, double *vz,
                    uint32_t *id, uint32_t *tc);
int o_set_particles(osim *o, int sp, int64_t n, const double *z, const double *vx,
                    const double *vy, const double *vz, const uint32_t *id, const uint32_t *tc);
void o_get_hist(const osim *o, int sp, int64_t *H);
void o_get_phi(const osim *o, double *phi);
void o_get_E(const osim *o, double *E);
void o_get_tally(const osim *o, otally *t);
void o_get_derived(const osim *o, oderived *d);

/* Boundary-flux and energy diagnostics from tallies over a window. */
typedef struct {
    double gamma_emit, gamma_emit_meas, gamma_ref, gamma_net, gamma_anode;
    double backflow_pct, eta_net, eta_anode;
    double gamma_abs[ONSP][2], q_abs[ONSP][2];
    double wf_eff, q_emit_theory, q_ion_cath_recomb, q_cool1, q_cool2;
    double q_ion_anode_recomb, q_anode1, q_anode2, phi_vc_eff;
} odiag;
void o_diag(double gamma_emit, double Tc, double w0, double window_s,
            const double count[ONSP][2], const double energy[ONSP][2], double n_emit,
            odiag *out);
double o_eta_vc(double phi_vc, double phi_w, double T_emit);

#ifdef __cplusplus
}
#endif
#endif
