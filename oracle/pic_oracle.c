/*
 * pic_oracle.c -- plain, slow, FP64 CPU oracle of the 1D3V electrostatic
 * PIC-MCC thermionic diode of Zhang, Zhou and Zhao (electron transpiration
 * cooling; helium cathode-anode diode).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code, header,
 * table or constant generator with the HIP path.
 *
 * The paper fixes WHAT a step computes (section "Model": numerical setup;
 * "Emission and collisions"; "Boundary energy diagnostics", eqs. 1-10) but
 * leaves the discretisation open.  Where it is silent this file follows the
 * readings listed in the design notes of the repository (CIC shape, leapfrog,
 * node-centred Dirichlet Poisson, flux-weighted emission, null-collision MCC
 * with isotropic centre-of-mass scattering, counter-based Philox draws keyed
 * by particle id).  Every floating-point quantity is double precision.
 *
 * Order of one step n (reading of "Model"; the paper gives no order):
 *   gather -> push -> absorb at the electrodes -> MCC -> births
 *   (ionisation, thermionic emission, pair replenishment) -> deposit -> solve.
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 exact / recommended values. */
#define Q_E 1.602176634e-19
#define K_B 1.380649e-23
#define EPS0 8.8541878128e-12
#define MASS_E 9.1093837015e-31
#define MASS_HE 6.6464731e-27
#define E_EXC 19.82   /* He excitation threshold (eV) */
#define E_ION 24.59   /* He first ionisation energy (eV), eqs. 3 and 7 */
#define TWO32 4294967296.0
#define PI_D 3.14159265358979323846

enum { EV_COLL = 1, EV_LOAD = 2, EV_EMIT = 3, EV_BIRTH = 4, EV_PROFILE = 5 };
#define LOAD_STEP 0xFFFFFFFFu
#define NEVER 0xFFFFFFFFu

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from its       */
/* published definition: ten rounds of two 32x32->64 multiplies with a       */
/* Weyl-sequence key schedule.                                               */
/* ------------------------------------------------------------------------ */
void o_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * x0;
        uint64_t p1 = (uint64_t)M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(uint32_t id, uint32_t kseed, uint32_t step, uint32_t ev, uint32_t sub,
                 uint32_t out[4])
{
    uint32_t ctr[4] = {step, ev, sub, 0u};
    uint32_t key[2] = {id, kseed};
    o_philox4x32_10(ctr, key, out);
}

/* Uniform mappings: every value is exactly representable, never 0 or 1. */
double o_u24(uint32_t w) { return (double)((w >> 9) * 2u + 1u) * (1.0 / 16777216.0); }
double o_u32(uint32_t w) { return ((double)w + 0.5) * (1.0 / TWO32); }
double o_u53(uint32_t hi, uint32_t lo)
{
    uint64_t m = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);   /* 52 bits */
    return ((double)m * 2.0 + 1.0) * (1.0 / 9007199254740992.0); /* / 2^53 */
}

/* Box-Muller pair from two 32-bit words. */
static void normal_pair32(uint32_t a, uint32_t b, double *n1, double *n2)
{
    double r = sqrt(-2.0 * log(o_u32(a)));
    double th = 2.0 * PI_D * o_u32(b);
    *n1 = r * cos(th);
    *n2 = r * sin(th);
}
/* Box-Muller pair on the 24-bit uniforms used by collision draws. */
static void normal_pair24(uint32_t a, uint32_t b, double *n1, double *n2)
{
    double r = sqrt(-2.0 * log(o_u24(a)));
    double th = 2.0 * PI_D * o_u24(b);
    *n1 = r * cos(th);
    *n2 = r * sin(th);
}

/* Number of steps to the next null-collision candidate: the free flight of
 * a Poisson process of rate numax (Vahedi-Surendra null collision), measured
 * in whole steps.  G >= 1.  lam = numax * dt. */
static uint32_t next_candidate(uint32_t base, double lam, uint32_t hi, uint32_t lo)
{
    if (!(lam > 0.0)) return NEVER;
    double g = ceil(-log(o_u53(hi, lo)) / lam);
    if (g < 1.0) g = 1.0;
    double t = (double)base + g;
    if (t >= 4294967295.0) return NEVER;
    return (uint32_t)t;
}

/* ------------------------------------------------------------------------ */
/* Cross sections ("Emission and collisions"; analytic forms for the         */
/* channels the paper takes from a database it does not print).             */
/* ------------------------------------------------------------------------ */
double o_sigma(const ocfg *c, int ch, double eps)
{
    if (!(c->channels & (1u << ch))) return 0.0;
    switch (ch) {
    case OCH_EEL: return c->sig_el;                 /* fixed effective e-He elastic */
    case OCH_EXC: {
        if (eps <= E_EXC) return 0.0;
        double x = eps / E_EXC;
        return c->sig_x0 * log(x) / x;
    }
    case OCH_IZ: {
        if (eps <= E_ION) return 0.0;
        return c->lotz_a * 2.0 * log(eps / E_ION) / (eps * E_ION);   /* Lotz, q = 2 */
    }
    case OCH_CX: return c->sig_cx;                  /* fixed effective He+-He CX */
    case OCH_IEL: return c->sig_iel;
    }
    return 0.0;
}

static double sigma_total(const ocfg *c, int ion, double eps)
{
    if (ion) return o_sigma(c, OCH_CX, eps) + o_sigma(c, OCH_IEL, eps);
    return o_sigma(c, OCH_EEL, eps) + o_sigma(c, OCH_EXC, eps) + o_sigma(c, OCH_IZ, eps);
}

/* Upper bound of n_g sigma_T(eps(g)) g over relative speeds up to a cap. */
static double nu_max(const ocfg *c, int ion, double m, double sig_n)
{
    if (!(c->ng > 0.0)) return 0.0;
    double mu = m * MASS_HE / (m + MASS_HE);
    double ecap = ion ? fabs(c->V) + 40.0 * c->Ti0 : fabs(c->V) + 40.0 * c->Te0 + 40.0 * c->Tc;
    double gcap = sqrt(2.0 * Q_E * ecap / m) + 6.0 * sig_n;
    double best = 0.0;
    for (int i = 1; i <= 65536; ++i) {
        double g = gcap * (double)i / 65536.0;
        double eps = 0.5 * mu * g * g / Q_E;
        double nu = c->ng * sigma_total(c, ion, eps) * g;
        if (nu > best) best = nu;
    }
    return best * 1.001;
}

int o_derive(const ocfg *c, oderived *d)
{
    if (c->N < 2 || !(c->L > 0.0) || c->n_load < 0 || !(c->dt > 0.0)) return -1;
    d->dz = c->L / (double)c->N;
    d->invdz = (double)c->N / c->L;
    d->w0 = c->n_load > 0 ? c->n0 * c->L / (double)c->n_load : 0.0;   /* w0 = n0 dz / Nppc */
    double mi = MASS_HE - MASS_E;
    d->mass[OSP_P] = MASS_E; d->mass[OSP_E] = MASS_E; d->mass[OSP_I] = mi;
    d->qm[OSP_P] = -Q_E / MASS_E; d->qm[OSP_E] = -Q_E / MASS_E; d->qm[OSP_I] = Q_E / mi;
    d->sig_n[0] = sqrt(Q_E * c->Tne / MASS_HE);
    d->sig_n[1] = sqrt(Q_E * c->Tni / MASS_HE);
    if (c->periodic) {
        d->numax[0] = d->numax[1] = 0.0;
    } else {
        d->numax[0] = nu_max(c, 0, MASS_E, d->sig_n[0]);
        d->numax[1] = nu_max(c, 1, mi, d->sig_n[1]);
    }
    d->lam[0] = d->numax[0] * c->dt;
    d->lam[1] = d->numax[1] * c->dt;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Particle storage                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *z, *vx, *vy, *vz;
    uint32_t *id, *tc;
    int64_t n, cap;
} ospecies;

typedef struct {
    uint32_t parent;
    int parent_sp;
    double z;
    double ve[3];   /* secondary electron */
    double vi[3];   /* new ion (the neutral's velocity) */
} oiz;

/* One particle's move in the step being taken: where the push put it, what
 * the walls and the collision did to it.  Filled for every particle before
 * any of them is tallied, so that the per-particle work can run on several
 * threads while the order-dependent work (tallies, ionisation products,
 * compaction) stays in particle order. */
typedef struct {
    double z;         /* position after the push */
    double vz_push;   /* v_z after the push, before any collision */
    double v[3];      /* velocity after the collision (= after the push if none) */
    uint32_t id, tc;
    int8_t fate;      /* 0 stays, 1 absorbed at the cathode, 2 at the anode */
    int8_t cand;      /* 1 if a null-collision candidate this step */
    int8_t ch;        /* channel taken, -1 none */
    double margin;    /* candidates: channel-choice margin (relative to nu_max) */
} omove;

struct osim {
    ocfg c;
    oderived d;
    ospecies sp[ONSP];
    int64_t *H[ONSP];
    double *rho, *phi, *E;
    int64_t step;
    uint32_t next_id;
    otally t;
    oiz *iz; int64_t niz, cap_iz;
    omove *mv[ONSP]; int64_t nmv[ONSP], cap_mv[ONSP];   /* the last step's moves per species */
};

static int sp_reserve(ospecies *s, int64_t need)
{
    if (need <= s->cap) return 0;
    int64_t cap = s->cap ? s->cap : 1024;
    while (cap < need) cap *= 2;
    double *z = realloc(s->z, cap * sizeof(double));
    double *vx = realloc(s->vx, cap * sizeof(double));
    double *vy = realloc(s->vy, cap * sizeof(double));
    double *vz = realloc(s->vz, cap * sizeof(double));
    uint32_t *id = realloc(s->id, cap * sizeof(uint32_t));
    uint32_t *tc = realloc(s->tc, cap * sizeof(uint32_t));
    if (z) s->z = z;
    if (vx) s->vx = vx;
    if (vy) s->vy = vy;
    if (vz) s->vz = vz;
    if (id) s->id = id;
    if (tc) s->tc = tc;
    if (!z || !vx || !vy || !vz || !id || !tc) return -1;
    s->cap = cap;
    return 0;
}

static int sp_push(ospecies *s, double z, double vx, double vy, double vz, uint32_t id, uint32_t tc)
{
    if (sp_reserve(s, s->n + 1)) return -1;
    s->z[s->n] = z; s->vx[s->n] = vx; s->vy[s->n] = vy; s->vz[s->n] = vz;
    s->id[s->n] = id; s->tc[s->n] = tc;
    s->n++;
    return 0;
}

osim *o_create(const ocfg *c)
{
    osim *o = calloc(1, sizeof(osim));
    if (!o) return NULL;
    o->c = *c;
    if (o_derive(c, &o->d)) { free(o); return NULL; }
    int nn = c->N + 1;
    for (int s = 0; s < ONSP; ++s) o->H[s] = calloc(nn, sizeof(int64_t));
    o->rho = calloc(nn, sizeof(double));
    o->phi = calloc(nn, sizeof(double));
    o->E = calloc(nn, sizeof(double));
    return o;
}

void o_destroy(osim *o)
{
    if (!o) return;
    for (int s = 0; s < ONSP; ++s) {
        free(o->sp[s].z); free(o->sp[s].vx); free(o->sp[s].vy); free(o->sp[s].vz);
        free(o->sp[s].id); free(o->sp[s].tc); free(o->H[s]); free(o->mv[s]);
    }
    free(o->rho); free(o->phi); free(o->E); free(o->iz);
    free(o);
}

/* ------------------------------------------------------------------------ */
/* Charge deposition: cloud-in-cell weights in 64-bit fixed point.          */
/* A particle at s = z/dz with j = floor(s), f = s - j adds 2^32 - a to     */
/* node j and a to node j+1, a = f * 2^32 rounded half-to-even, so every   */
/* particle deposits exactly 2^32 and the sum is order independent.        */
/* ------------------------------------------------------------------------ */
static void cic(double z, int32_t N, double invdz, int32_t *j, double *f)
{
    double s = z * invdz;
    double fl = floor(s);
    int32_t jj = (int32_t)fl;
    if (jj < 0) { jj = 0; fl = 0.0; }
    if (jj > N - 1) { jj = N - 1; fl = (double)(N - 1); }
    *j = jj;
    *f = s - fl;
}

void o_deposit(int64_t n, const double *z, int32_t N, double invdz, int64_t *H)
{
    /* integer sums: any split over threads gives the same histogram */
#pragma omp parallel for schedule(static) reduction(+ : H[0 : N + 1])
    for (int64_t p = 0; p < n; ++p) {
        int32_t j; double f;
        cic(z[p], N, invdz, &j, &f);
        int64_t a = (int64_t)nearbyint(f * TWO32);
        H[j] += (int64_t)4294967296LL - a;
        H[j + 1] += a;
    }
}

static void deposit_periodic(int64_t n, const double *z, int32_t N, double invdz, int64_t *H)
{
    for (int64_t p = 0; p < n; ++p) {
        int32_t j; double f;
        cic(z[p], N, invdz, &j, &f);
        int64_t a = (int64_t)nearbyint(f * TWO32);
        H[j] += (int64_t)4294967296LL - a;
        H[(j + 1) % N] += a;
    }
}

/* ------------------------------------------------------------------------ */
/* Poisson: phi_{j-1} - 2 phi_j + phi_{j+1} = -rho_j dz^2 / eps0 on the     */
/* interior nodes, phi_0 = 0 (cathode), phi_N = V (anode)                   */
/* ("Model": potential from the charge density every step, Dirichlet        */
/* electrodes).  Solved by the Thomas algorithm.                            */
/* ------------------------------------------------------------------------ */
int o_solve(int32_t N, double dz, double V, const double *rho, double *phi)
{
    int n = N - 1;                       /* unknowns phi_1 .. phi_{N-1} */
    phi[0] = 0.0;
    phi[N] = V;
    if (n <= 0) return 0;
    double *cp = malloc(n * sizeof(double));
    double *dp = malloc(n * sizeof(double));
    if (!cp || !dp) { free(cp); free(dp); return -1; }
    /* row i (node j = i+1): a = 1, b = -2, c = 1, rhs = -rho dz^2/eps0 - boundary terms */
    for (int i = 0; i < n; ++i) {
        int j = i + 1;
        double rhs = -rho[j] * dz * dz / EPS0;
        if (j == 1) rhs -= phi[0];
        if (j == N - 1) rhs -= phi[N];
        double a = (i > 0) ? 1.0 : 0.0, b = -2.0, cc = (i < n - 1) ? 1.0 : 0.0;
        if (i == 0) {
            cp[i] = cc / b;
            dp[i] = rhs / b;
        } else {
            double m = b - a * cp[i - 1];
            cp[i] = cc / m;
            dp[i] = (rhs - a * dp[i - 1]) / m;
        }
    }
    phi[n] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) phi[i + 1] = dp[i] - cp[i] * phi[i + 2];
    free(cp);
    free(dp);
    return 0;
}

/* E = -dphi/dz: central difference inside, one-sided at the electrodes. */
void o_efield(int32_t N, double dz, const double *phi, double *E)
{
    for (int j = 1; j < N; ++j) E[j] = (phi[j - 1] - phi[j + 1]) / (2.0 * dz);
    E[0] = (phi[0] - phi[1]) / dz;
    E[N] = (phi[N - 1] - phi[N]) / dz;
}

static void field_nonperiodic(osim *o)
{
    const ocfg *c = &o->c;
    int nn = c->N + 1;
    double k = Q_E * o->d.w0 / (TWO32 * o->d.dz);
    for (int j = 0; j < nn; ++j) {
        int64_t R = o->H[OSP_I][j] - o->H[OSP_P][j] - o->H[OSP_E][j];
        o->rho[j] = k * (double)R;
    }
    o_solve(c->N, o->d.dz, c->V, o->rho, o->phi);
    o_efield(c->N, o->d.dz, o->phi, o->E);
}

/* Periodic test mode: nodes 0..N-1 (node N is node 0), neutralising
 * background (mean of rho removed), gauge phi_0 = 0. */
static void field_periodic(osim *o)
{
    const ocfg *c = &o->c;
    int N = c->N;
    double k = Q_E * o->d.w0 / (TWO32 * o->d.dz);
    double mean = 0.0;
    for (int j = 0; j < N; ++j) {
        int64_t R = o->H[OSP_I][j] - o->H[OSP_P][j] - o->H[OSP_E][j];
        o->rho[j] = k * (double)R;
        mean += o->rho[j];
    }
    mean /= (double)N;
    for (int j = 0; j < N; ++j) o->rho[j] -= mean;
    o->rho[N] = o->rho[0];
    /* With zero net charge the cyclic system is consistent; pinning phi_0 =
     * phi_N = 0 and solving nodes 1..N-1 satisfies the equation at node 0 too. */
    o_solve(N, o->d.dz, 0.0, o->rho, o->phi);
    for (int j = 0; j < N; ++j) {
        int jm = (j + N - 1) % N, jp = (j + 1) % N;
        o->E[j] = (o->phi[jm] - o->phi[jp]) / (2.0 * o->d.dz);
    }
    o->E[N] = o->E[0];
}

int o_refield(osim *o)
{
    const ocfg *c = &o->c;
    int nn = c->N + 1;
    for (int s = 0; s < ONSP; ++s) {
        memset(o->H[s], 0, nn * sizeof(int64_t));
        if (c->periodic)
            deposit_periodic(o->sp[s].n, o->sp[s].z, c->N, o->d.invdz, o->H[s]);
        else
            o_deposit(o->sp[s].n, o->sp[s].z, c->N, o->d.invdz, o->H[s]);
    }
    if (c->periodic) field_periodic(o); else field_nonperiodic(o);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Initial load ("Model": uniform positions, Maxwellian velocities at Te0,  */
/* Ti0, zero drift).  Plasma electrons get ids 0..n_load-1, ions           */
/* n_load..2 n_load-1.                                                      */
/* ------------------------------------------------------------------------ */
static uint32_t kseed(const osim *o) { return o->c.seed ^ o->c.diode; }

int o_load(osim *o)
{
    const ocfg *c = &o->c;
    for (int s = 0; s < ONSP; ++s) o->sp[s].n = 0;
    memset(&o->t, 0, sizeof(o->t));
    o->step = 0;
    uint32_t id = 0;
    const int load_sp[2] = {OSP_P, OSP_I};
    for (int q = 0; q < 2; ++q) {
        int s = load_sp[q];
        double T = (s == OSP_I) ? c->Ti0 : c->Te0;
        double sig = sqrt(Q_E * T / o->d.mass[s]);
        double lam = o->d.lam[s == OSP_I ? 1 : 0];
        ospecies *S = &o->sp[s];
        if (sp_reserve(S, c->n_load)) return -1;
        /* particle p of the species has id id0 + p and its own draws */
        const uint32_t id0 = id;
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < c->n_load; ++p) {
            const uint32_t pid = id0 + (uint32_t)p;
            uint32_t b0[4], b1[4];
            draw(pid, kseed(o), LOAD_STEP, EV_LOAD, 0, b0);
            draw(pid, kseed(o), LOAD_STEP, EV_LOAD, 1, b1);
            double n1, n2, n3, n4;
            normal_pair32(b0[0], b0[1], &n1, &n2);
            normal_pair32(b0[2], b0[3], &n3, &n4);
            /* first candidate step: the first whole step of the free flight */
            uint32_t tc = next_candidate(0u, lam, b1[2], b1[3]);
            if (tc != NEVER) tc -= 1u;
            S->z[p] = c->L * o_u53(b1[0], b1[1]);
            S->vx[p] = sig * n1; S->vy[p] = sig * n2; S->vz[p] = sig * n3;
            S->id[p] = pid; S->tc[p] = tc;
        }
        S->n = c->n_load;
        id += (uint32_t)c->n_load;
    }
    o->next_id = id;
    return o_refield(o);
}

/* Warm start from density profiles (a loaded state whose densities follow
 * given n_e(z), n_i(z) at the N cell centres instead of the uniform n0).
 * Cell j of species q (0: electrons, 1: ions) receives floor(x) particles
 * plus one with probability frac(x), x = n_q[j] dz / w0; the Bernoulli draw
 * is keyed by the cell: key (j, seed ^ diode), counter (LOAD, PROFILE, q, 0).
 * Ids run over the electron cells in order, then the ion cells.  Each
 * particle then draws exactly as in the uniform load, except that its
 * position is uniform inside its cell: z = (j + U) dz. */
int o_load_profiles(osim *o, const double *ne, const double *ni)
{
    const ocfg *c = &o->c;
    for (int s = 0; s < ONSP; ++s) o->sp[s].n = 0;
    memset(&o->t, 0, sizeof(o->t));
    o->step = 0;
    uint32_t id = 0;
    const int load_sp[2] = {OSP_P, OSP_I};
    for (int q = 0; q < 2; ++q) {
        const int s = load_sp[q];
        const double *dens = q == 0 ? ne : ni;
        const double T = (s == OSP_I) ? c->Ti0 : c->Te0;
        const double sig = sqrt(Q_E * T / o->d.mass[s]);
        const double lam = o->d.lam[s == OSP_I ? 1 : 0];
        for (int32_t j = 0; j < c->N; ++j) {
            const double x = dens[j] * o->d.dz / o->d.w0;
            if (!(x >= 0.0) || x > 1073741824.0) return -2;
            const double fl = floor(x);
            uint32_t bc[4];
            draw((uint32_t)j, kseed(o), LOAD_STEP, EV_PROFILE, (uint32_t)q, bc);
            const int64_t cnt = (int64_t)fl + (o_u53(bc[0], bc[1]) < x - fl ? 1 : 0);
            if (sp_reserve(&o->sp[s], o->sp[s].n + cnt)) return -1;
            for (int64_t p = 0; p < cnt; ++p, ++id) {
                uint32_t b0[4], b1[4];
                draw(id, kseed(o), LOAD_STEP, EV_LOAD, 0, b0);
                draw(id, kseed(o), LOAD_STEP, EV_LOAD, 1, b1);
                double n1, n2, n3, n4;
                normal_pair32(b0[0], b0[1], &n1, &n2);
                normal_pair32(b0[2], b0[3], &n3, &n4);
                const double z = ((double)j + o_u53(b1[0], b1[1])) * o->d.dz;
                uint32_t tc = next_candidate(0u, lam, b1[2], b1[3]);
                if (tc != NEVER) tc -= 1u;
                sp_push(&o->sp[s], z, sig * n1, sig * n2, sig * n3, id, tc);
            }
        }
    }
    o->next_id = id;
    return o_refield(o);
}

/* Warm start with velocity distributions (a reading: the paper starts every
 * run from a uniform Maxwellian plasma).  A late-time run's particles in one
 * cell are summarised per species by quantiles of v_z and of the transverse
 * speed |v_perp| at nine levels; a loaded particle draws each from the
 * piecewise-linear inverse of its cell's quantile function and a uniform
 * azimuth for (v_x, v_y).  The quantiles are first sorted (monotone
 * rearrangement).  A kinetic energy above the null-collision bound's energy
 * cap (the energy up to which the bound was scanned) is scaled down to it. */
static const double OQ_LEVELS[OQ] = {0.0, 0.02, 0.1, 0.25, 0.5, 0.75, 0.9, 0.98, 1.0};

static void sort9(double q[OQ])
{
    for (int a = 1; a < OQ; ++a)
        for (int b = a; b > 0 && q[b - 1] > q[b]; --b) {
            double t = q[b];
            q[b] = q[b - 1];
            q[b - 1] = t;
        }
}

static double inv_quantile(const double q[OQ], double u)
{
    int k = 0;
    while (k < OQ - 2 && u >= OQ_LEVELS[k + 1]) ++k;
    double t = (u - OQ_LEVELS[k]) / (OQ_LEVELS[k + 1] - OQ_LEVELS[k]);
    return q[k] + t * (q[k + 1] - q[k]);
}

int o_load_state(osim *o, const double *prof)
{
    const ocfg *c = &o->c;
    const int64_t N = c->N;
    for (int64_t r = 0; r < OSTATE_ROWS * N; ++r)
        if (!isfinite(prof[r])) return -2;
    for (int s = 0; s < ONSP; ++s) o->sp[s].n = 0;
    memset(&o->t, 0, sizeof(o->t));
    o->step = 0;
    uint32_t id = 0;
    const int load_sp[2] = {OSP_P, OSP_I};
    for (int q = 0; q < 2; ++q) {
        const int s = load_sp[q];
        const double *dens = prof + (int64_t)q * N;
        const double lam = o->d.lam[q];
        const double m = o->d.mass[s];
        /* the null-collision bound's energy cap (eV) */
        const double cap = q ? fabs(c->V) + 40.0 * c->Ti0 : fabs(c->V) + 40.0 * c->Te0 + 40.0 * c->Tc;
        for (int32_t j = 0; j < c->N; ++j) {
            const double x = dens[j] * o->d.dz / o->d.w0;
            if (!(x >= 0.0) || x > 1073741824.0) return -2;
            double qz[OQ], qp[OQ];
            for (int k = 0; k < OQ; ++k) {
                qz[k] = prof[(int64_t)(3 + 18 * q + k) * N + j];
                qp[k] = prof[(int64_t)(12 + 18 * q + k) * N + j];
            }
            sort9(qz);
            sort9(qp);
            const double emax = Q_E * cap;     /* J */
            const double fl = floor(x);
            uint32_t bc[4];
            draw((uint32_t)j, kseed(o), LOAD_STEP, EV_PROFILE, (uint32_t)q, bc);
            const int64_t cnt = (int64_t)fl + (o_u53(bc[0], bc[1]) < x - fl ? 1 : 0);
            if (sp_reserve(&o->sp[s], o->sp[s].n + cnt)) return -1;
            for (int64_t p = 0; p < cnt; ++p, ++id) {
                uint32_t b0[4], b1[4], b2[4];
                draw(id, kseed(o), LOAD_STEP, EV_LOAD, 0, b0);
                draw(id, kseed(o), LOAD_STEP, EV_LOAD, 1, b1);
                draw(id, kseed(o), LOAD_STEP, EV_LOAD, 2, b2);
                double vz = inv_quantile(qz, o_u53(b0[0], b0[1]));
                double vp = fmax(0.0, inv_quantile(qp, o_u53(b0[2], b0[3])));
                const double az = 2.0 * PI_D * o_u53(b2[0], b2[1]);
                double vx = vp * cos(az), vy = vp * sin(az);
                const double e = 0.5 * m * (vx * vx + vy * vy + vz * vz);
                if (e > emax) {
                    const double f = emax > 0.0 ? sqrt(emax / e) : 0.0;
                    vx *= f;
                    vy *= f;
                    vz *= f;
                }
                const double z = ((double)j + o_u53(b1[0], b1[1])) * o->d.dz;
                uint32_t tc = next_candidate(0u, lam, b1[2], b1[3]);
                if (tc != NEVER) tc -= 1u;
                sp_push(&o->sp[s], z, vx, vy, vz, id, tc);
            }
        }
    }
    o->next_id = id;
    return o_refield(o);
}

/* ------------------------------------------------------------------------ */
/* MCC ("Emission and collisions": Monte Carlo collisions with a uniform    */
/* helium background; the neutral target velocity is drawn from a           */
/* Maxwellian at the prescribed neutral temperature).                       */
/* ------------------------------------------------------------------------ */
static void iso_dir(uint32_t wc, uint32_t wp, double d[3])
{
    double ct = 1.0 - 2.0 * o_u24(wc);
    double ph = 2.0 * PI_D * o_u24(wp);
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    d[0] = st * cos(ph);
    d[1] = st * sin(ph);
    d[2] = ct;
}

/* Returns the channel taken (-1 null).  v (3) is updated in place.  For
 * ionisation the secondary electron and new ion velocities are returned. */
static int mcc(const osim *o, int sp, uint32_t id, uint32_t n, double v[3], double ve[3], double vi[3],
               uint32_t *tc, int *exceeded, double *margin)
{
    const ocfg *c = &o->c;
    const oderived *d = &o->d;
    int ion = (sp == OSP_I);
    double m = d->mass[sp];
    double mu = m * MASS_HE / (m + MASS_HE);
    uint32_t C0[4], C1[4], C2[4];
    draw(id, kseed(o), n, EV_COLL, 0, C0);
    draw(id, kseed(o), n, EV_COLL, 1, C1);
    draw(id, kseed(o), n, EV_COLL, 2, C2);
    double sn = d->sig_n[ion];
    double a1, a2, a3, a4;
    normal_pair24(C0[0], C0[1], &a1, &a2);
    normal_pair24(C0[2], C0[3], &a3, &a4);
    double vn[3] = {sn * a1, sn * a2, sn * a3};
    double g[3] = {v[0] - vn[0], v[1] - vn[1], v[2] - vn[2]};
    double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    double gm = sqrt(g2);
    double eps = 0.5 * mu * g2 / Q_E;
    /* channel frequencies nu_k = n_g sigma_k(eps) |g|, fixed order */
    int chs[3]; int nch = 0;
    if (ion) { chs[nch++] = OCH_CX; chs[nch++] = OCH_IEL; }
    else { chs[nch++] = OCH_EEL; chs[nch++] = OCH_EXC; chs[nch++] = OCH_IZ; }
    double numax = d->numax[ion];
    double r = o_u24(C1[0]) * numax;
    double cum = 0.0;
    int taken = -1;
    /* margin: distance of r from the nearest cumulative boundary, relative
     * to numax (how close the channel choice came to another outcome) */
    double mg = INFINITY;
    for (int q = 0; q < nch; ++q) {
        cum += c->ng * o_sigma(c, chs[q], eps) * gm;
        if (taken < 0 && r < cum) taken = chs[q];
        if (fabs(r - cum) < mg) mg = fabs(r - cum);
    }
    *margin = numax > 0.0 ? mg / numax : INFINITY;
    *exceeded = cum > numax;
    *tc = next_candidate(n, d->lam[ion], C2[2], C2[3]);
    if (taken < 0) return -1;

    double M = MASS_HE;
    double vcm[3], dir[3];
    for (int k = 0; k < 3; ++k) vcm[k] = (m * v[k] + M * vn[k]) / (m + M);
    double fr = M / (m + M);
    if (taken == OCH_CX) {
        /* charge exchange: the ion leaves with the neutral's velocity */
        for (int k = 0; k < 3; ++k) v[k] = vn[k];
        return taken;
    }
    iso_dir(C1[1], C1[2], dir);
    if (taken == OCH_EEL || taken == OCH_IEL) {
        for (int k = 0; k < 3; ++k) v[k] = vcm[k] + fr * gm * dir[k];
        return taken;
    }
    if (taken == OCH_EXC) {
        double gp2 = g2 - 2.0 * Q_E * E_EXC / mu;
        double gp = sqrt(fmax(0.0, gp2));
        for (int k = 0; k < 3; ++k) v[k] = vcm[k] + fr * gp * dir[k];
        return taken;
    }
    /* ionisation: the energy above threshold is shared at random between the
     * scattered and the secondary electron; the new ion carries the neutral's
     * velocity */
    double avail = eps - E_ION;
    if (avail < 0.0) avail = 0.0;
    double e1 = o_u24(C1[3]) * avail;
    double e2 = avail - e1;
    double g1 = sqrt(2.0 * Q_E * e1 / mu);
    double gs = sqrt(2.0 * Q_E * e2 / mu);
    double dir2[3];
    iso_dir(C2[0], C2[1], dir2);
    for (int k = 0; k < 3; ++k) {
        v[k] = vcm[k] + fr * g1 * dir[k];
        ve[k] = vcm[k] + fr * gs * dir2[k];
        vi[k] = vn[k];
    }
    return taken;
}

static int cmp_iz(const void *a, const void *b)
{
    uint32_t x = ((const oiz *)a)->parent, y = ((const oiz *)b)->parent;
    return (x > y) - (x < y);
}

static void tally_abs(osim *o, int sp, int wall, double vx, double vy, double vz)
{
    o->t.abs_count[sp][wall]++;
    o->t.abs_energy[sp][wall] += 0.5 * o->d.mass[sp] * (vx * vx + vy * vy + vz * vz);
}

/* Births draw from their own id: B0 = (n, EV_BIRTH, 0), B1 = (n, EV_BIRTH, 1). */
static int birth(osim *o, int sp, uint32_t id, double z, double vx, double vy, double vz)
{
    const ocfg *c = &o->c;
    uint32_t b1[4];
    draw(id, kseed(o), (uint32_t)o->step, EV_BIRTH, 1, b1);
    uint32_t tc = next_candidate((uint32_t)o->step, o->d.lam[sp == OSP_I ? 1 : 0], b1[2], b1[3]);
    if (z <= 0.0) { tally_abs(o, sp, 0, vx, vy, vz); return 0; }
    if (z >= c->L) { tally_abs(o, sp, 1, vx, vy, vz); return 0; }
    return sp_push(&o->sp[sp], z, vx, vy, vz, id, tc);
}

int o_step(osim *o)
{
    const ocfg *c = &o->c;
    const oderived *d = &o->d;
    uint32_t n = (uint32_t)o->step;
    int64_t ion_lost = 0;
    o->niz = 0;

    for (int sp = 0; sp < ONSP; ++sp) {
        ospecies *s = &o->sp[sp];
        const int ion = (sp == OSP_I);
        if (s->n > o->cap_mv[sp]) {
            omove *m = realloc(o->mv[sp], s->n * sizeof(omove));
            if (!m) return -1;
            o->mv[sp] = m;
            o->cap_mv[sp] = s->n;
        }
        omove *mv = o->mv[sp];
        o->nmv[sp] = s->n;
        int64_t exceed = 0;
        /* per particle: gather, push, wall test, collision */
#pragma omp parallel for schedule(static) reduction(+ : exceed)
        for (int64_t p = 0; p < s->n; ++p) {
            omove *m = &mv[p];
            /* gather (CIC, same weights as the deposit) */
            int32_t j; double f;
            cic(s->z[p], c->N, d->invdz, &j, &f);
            int32_t j1 = c->periodic ? (j + 1) % c->N : j + 1;
            double Ep = (1.0 - f) * o->E[j] + f * o->E[j1];
            /* leapfrog: v^{n+1/2} = v^{n-1/2} + (q/m) E dt ; z^{n+1} = z^n + v dt */
            double vz = s->vz[p] + d->qm[sp] * Ep * c->dt;
            double z = s->z[p] + vz * c->dt;
            m->id = s->id[p];
            m->tc = s->tc[p];
            m->vz_push = vz;
            m->v[0] = s->vx[p]; m->v[1] = s->vy[p]; m->v[2] = vz;
            m->cand = 0; m->ch = -1; m->margin = INFINITY; m->fate = 0;
            if (c->periodic) {
                while (z < 0.0) z += c->L;
                while (z >= c->L) z -= c->L;
            } else if (z <= 0.0 || z >= c->L) {
                m->fate = z <= 0.0 ? 1 : 2;   /* absorbing electrodes */
            } else if (m->tc == n) {
                double ve[3], vi[3];
                int ex = 0;
                m->cand = 1;
                m->ch = (int8_t)mcc(o, sp, m->id, n, m->v, ve, vi, &m->tc, &ex, &m->margin);
                exceed += ex;
            }
            m->z = z;
        }
        o->t.nullcoll_exceed += exceed;
        /* in particle order: tallies, ionisation events, compaction */
        int64_t keep = 0;
        for (int64_t p = 0; p < s->n; ++p) {
            const omove *m = &mv[p];
            if (m->fate) {
                tally_abs(o, sp, m->fate - 1, m->v[0], m->v[1], m->v[2]);
                if (ion) ion_lost++;
                continue;
            }
            if (m->cand) {
                o->t.cand[ion]++;
                if (m->ch >= 0) o->t.coll[m->ch]++;
                if (m->ch == OCH_IZ) {
                    /* the products: the same (pure) collision once more from the
                     * pre-collision velocity */
                    double v[3] = {s->vx[p], s->vy[p], m->vz_push}, ve[3], vi[3];
                    uint32_t tc2;
                    int ex;
                    double mg;
                    mcc(o, sp, m->id, n, v, ve, vi, &tc2, &ex, &mg);
                    if (o->niz == o->cap_iz) {
                        int64_t nc = o->cap_iz ? 2 * o->cap_iz : 64;
                        oiz *t = realloc(o->iz, nc * sizeof(oiz));
                        if (!t) return -1;
                        o->iz = t; o->cap_iz = nc;
                    }
                    oiz *e = &o->iz[o->niz++];
                    e->parent = m->id; e->parent_sp = sp; e->z = m->z;
                    for (int k = 0; k < 3; ++k) { e->ve[k] = ve[k]; e->vi[k] = vi[k]; }
                }
            }
            s->z[keep] = m->z; s->vx[keep] = m->v[0]; s->vy[keep] = m->v[1]; s->vz[keep] = m->v[2];
            s->id[keep] = m->id; s->tc[keep] = m->tc;
            keep++;
        }
        s->n = keep;
    }

    if (!c->periodic) {
        /* ionisation products, in increasing parent id */
        qsort(o->iz, o->niz, sizeof(oiz), cmp_iz);
        for (int64_t r = 0; r < o->niz; ++r) {
            oiz *e = &o->iz[r];
            uint32_t ide = o->next_id++, idi = o->next_id++;
            if (birth(o, OSP_P, ide, e->z, e->ve[0], e->ve[1], e->ve[2])) return -1;
            if (birth(o, OSP_I, idi, e->z, e->vi[0], e->vi[1], e->vi[2])) return -1;
        }
        o->t.n_iz += o->niz;

        /* thermionic emission ("Emission and collisions"): N_emit = Gamma dt / w0
         * with a Bernoulli draw for the fractional part; flux-weighted
         * half-Maxwellian at Tc; placed at z = v_z dt. */
        if (c->gamma_emit > 0.0 && d->w0 > 0.0) {
            double x = c->gamma_emit * c->dt / d->w0;
            double fl = floor(x);
            uint32_t be[4];
            draw(0xFFFFFFFFu, kseed(o), n, EV_EMIT, 0, be);
            int64_t ne = (int64_t)fl + (o_u53(be[0], be[1]) < (x - fl) ? 1 : 0);
            double sc = sqrt(Q_E * c->Tc / MASS_E);
            for (int64_t i = 0; i < ne; ++i) {
                uint32_t idn = o->next_id++;
                uint32_t b0[4];
                draw(idn, kseed(o), n, EV_BIRTH, 0, b0);
                double n1, n2;
                normal_pair32(b0[0], b0[1], &n1, &n2);
                double vz = sc * sqrt(-2.0 * log(o_u53(b0[2], b0[3])));
                if (birth(o, OSP_E, idn, vz * c->dt, sc * n1, sc * n2, vz)) return -1;
            }
            o->t.n_emit += ne;
        }

        /* pair replenishment ("Model"): as many e-ion pairs as ions were lost
         * this step, at a shared uniform position, Maxwellian at Te0 / Ti0 */
        if (c->replenish) {
            double se = sqrt(Q_E * c->Te0 / MASS_E), si = sqrt(Q_E * c->Ti0 / d->mass[OSP_I]);
            for (int64_t r = 0; r < ion_lost; ++r) {
                uint32_t ide = o->next_id++, idi = o->next_id++;
                uint32_t e0[4], e1[4], i0[4];
                draw(ide, kseed(o), n, EV_BIRTH, 0, e0);
                draw(ide, kseed(o), n, EV_BIRTH, 1, e1);
                draw(idi, kseed(o), n, EV_BIRTH, 0, i0);
                double z = c->L * o_u53(e1[0], e1[1]);
                double a1, a2, a3, a4;
                normal_pair32(e0[0], e0[1], &a1, &a2);
                normal_pair32(e0[2], e0[3], &a3, &a4);
                if (birth(o, OSP_P, ide, z, se * a1, se * a2, se * a3)) return -1;
                normal_pair32(i0[0], i0[1], &a1, &a2);
                normal_pair32(i0[2], i0[3], &a3, &a4);
                if (birth(o, OSP_I, idi, z, si * a1, si * a2, si * a3)) return -1;
            }
            o->t.n_repl += ion_lost;
        }
    }

    o->step++;
    return o_refield(o);
}

/* ------------------------------------------------------------------------ */
/* Accessors                                                                */
/* ------------------------------------------------------------------------ */
int64_t o_count(const osim *o, int sp) { return o->sp[sp].n; }

/* Threads this build runs the per-particle loops on (1 without OpenMP). */
int o_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}

int64_t o_last_moves_count(const osim *o, int sp) { return o->nmv[sp]; }

/* The last step's moves of one species, in the particle order of that step:
 * id, position after the push, fate (0 stays, 1 cathode, 2 anode), channel
 * (-1 none; -2 not a candidate) and the channel-choice margin of candidates.
 * Returns the count (arrays must hold o_count before the step). */
int64_t o_last_moves(const osim *o, int sp, uint32_t *id, double *z, int32_t *fate, int32_t *ch,
                     double *margin)
{
    for (int64_t p = 0; p < o->nmv[sp]; ++p) {
        const omove *m = &o->mv[sp][p];
        id[p] = m->id;
        z[p] = m->z;
        fate[p] = m->fate;
        ch[p] = m->cand ? m->ch : -2;
        margin[p] = m->margin;
    }
    return o->nmv[sp];
}
int64_t o_stepno(const osim *o) { return o->step; }
uint32_t o_next_id(const osim *o) { return o->next_id; }
void o_set_counters(osim *o, int64_t step, uint32_t next_id) { o->step = step; o->next_id = next_id; }

int o_get_particles(const osim *o, int sp, double *z, double *vx, double *vy, double *vz,
                    uint32_t *id, uint32_t *tc)
{
    const ospecies *s = &o->sp[sp];
    for (int64_t p = 0; p < s->n; ++p) {
        if (z) z[p] = s->z[p];
        if (vx) vx[p] = s->vx[p];
        if (vy) vy[p] = s->vy[p];
        if (vz) vz[p] = s->vz[p];
        if (id) id[p] = s->id[p];
        if (tc) tc[p] = s->tc[p];
    }
    return 0;
}

int o_set_particles(osim *o, int sp, int64_t n, const double *z, const double *vx,
                    const double *vy, const double *vz, const uint32_t *id, const uint32_t *tc)
{
    ospecies *s = &o->sp[sp];
    if (sp_reserve(s, n)) return -1;
    for (int64_t p = 0; p < n; ++p) {
        s->z[p] = z[p]; s->vx[p] = vx[p]; s->vy[p] = vy[p]; s->vz[p] = vz[p];
        s->id[p] = id[p]; s->tc[p] = tc[p];
    }
    s->n = n;
    return 0;
}

void o_get_hist(const osim *o, int sp, int64_t *H) { memcpy(H, o->H[sp], (o->c.N + 1) * sizeof(int64_t)); }
void o_get_phi(const osim *o, double *phi) { memcpy(phi, o->phi, (o->c.N + 1) * sizeof(double)); }
void o_get_E(const osim *o, double *E) { memcpy(E, o->E, (o->c.N + 1) * sizeof(double)); }
void o_get_tally(const osim *o, otally *t) { *t = o->t; }
void o_get_derived(const osim *o, oderived *d) { *d = o->d; }

/* ------------------------------------------------------------------------ */
/* Diagnostics ("Benchmark cases" and "Boundary energy diagnostics")        */
/* ------------------------------------------------------------------------ */
void o_diag(double gamma_emit, double Tc, double w0, double window_s,
            const double count[ONSP][2], const double energy[ONSP][2], double n_emit,
            odiag *out)
{
    memset(out, 0, sizeof(*out));
    double inv = w0 / window_s;
    for (int s = 0; s < ONSP; ++s)
        for (int w = 0; w < 2; ++w) {
            out->gamma_abs[s][w] = count[s][w] * inv;
            out->q_abs[s][w] = energy[s][w] * inv;
        }
    out->gamma_emit = gamma_emit;
    out->gamma_emit_meas = n_emit * inv;
    /* Gamma_net = Gamma_emit - Gamma_ref; backflow ratio = Gamma_ref/Gamma_emit */
    out->gamma_ref = out->gamma_abs[OSP_E][0];
    out->gamma_anode = out->gamma_abs[OSP_E][1];
    out->gamma_net = gamma_emit - out->gamma_ref;
    out->backflow_pct = 100.0 * out->gamma_ref / gamma_emit;
    out->eta_net = out->gamma_net / gamma_emit;
    out->eta_anode = out->gamma_anode / gamma_emit;
    /* eq. 2: W_F,eff = -Tc ln[e Gamma / (A_R Tc^2)], A_R = 1.20e6/(k_B/e)^2 */
    double kbe = K_B / Q_E;
    double AR = 1.20e6 / (kbe * kbe);
    out->wf_eff = -Tc * log(Q_E * gamma_emit / (AR * Tc * Tc));
    /* eq. 1 */
    out->q_emit_theory = gamma_emit * Q_E * (out->wf_eff + 2.0 * Tc);
    /* eq. 3 */
    out->q_ion_cath_recomb = out->gamma_abs[OSP_I][0] * Q_E * E_ION;
    /* eqs. 4, 5 */
    out->q_cool1 = out->q_emit_theory - out->q_abs[OSP_E][0] - out->q_abs[OSP_P][0] - out->q_abs[OSP_I][0];
    out->q_cool2 = out->q_cool1 - out->q_ion_cath_recomb;
    /* eqs. 6-8 */
    out->q_anode1 = out->q_abs[OSP_E][1] + out->q_abs[OSP_P][1] + out->q_abs[OSP_I][1];
    out->q_ion_anode_recomb = out->gamma_abs[OSP_I][1] * Q_E * E_ION;
    out->q_anode2 = out->q_anode1 + out->q_ion_anode_recomb;
    /* eq. 10 */
    out->phi_vc_eff = out->gamma_net > 0.0 ? Tc * log(out->gamma_net / gamma_emit) : NAN;
}

/* eq. 9 */
double o_eta_vc(double phi_vc, double phi_w, double T_emit) { return exp((phi_vc - phi_w) / T_emit); }
