// pic_host.hip -- host side of the C ABI declared in include/pic.h.
//
// Configuration derivation, workspace layout, launch schedule (load, cell
// re-sort every K steps, particle kernel, sources+field kernel), and the
// host-side diagnostics of "Benchmark cases" / "Boundary energy diagnostics"
// (eqs. 1-10) computed from the device's integer tallies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/pic.h"
#include "pic_internal.h"

using namespace pic;

extern "C" hipError_t picx_launch_load(const Diode *D, const long long *n_load, int nd, long long max_load,
                                       hipStream_t s);
extern "C" hipError_t picx_launch_particles(const Diode *D, DiodeState *S, int nd, int mode, int ppt, int grid,
                                            int parity, hipStream_t s);
extern "C" hipError_t picx_launch_sources_field(const Diode *D, DiodeState *S, int nd, int mode, int max_nodes,
                                                int parity, hipStream_t s);
extern "C" hipError_t picx_prepare(void);
extern "C" hipError_t picx_launch_phase_hist(const Diode *D, const DiodeState *S, int d, int s, int parity, int nz,
                                             int nv, double sz, double vmin, double sv, unsigned long long *out,
                                             int blocks, hipStream_t st);
extern "C" int picx_sources_field_kernels(int max_nodes, int mode);
extern "C" hipError_t picx_launch_profile_load(const Diode *D, const double *dens, int rows, int nd, int max_cells,
                                               hipStream_t s);
extern "C" hipError_t picx_launch_sort(const Diode *D, DiodeState *S, int nd, int ppt, int grid, int parity,
                                       hipStream_t s);

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(PIC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;
constexpr int TPOS = 8;   // particle kernels timed per replayed graph (pic_step_timed)
constexpr size_t GRAPH_CACHE = 16;   // captured step runs kept per handle
constexpr int64_t TIMED_MAX = 4096;   // particle kernels timed per pic_step_timed call
constexpr int64_t PLAIN_SAMPLES = 32; // of them, at most, on the plain stream

// ----------------------------------------------------------------------------
// Derived quantities ("Model": w0 = n0 dz / N_ppc, dt and grid; MCC bound).
// ----------------------------------------------------------------------------
double sigma_ch(const pic_config &c, int ch, double eps)
{
    if (!(c.channels & (1u << ch))) return 0.0;
    switch (ch) {
    case CH_EEL: return c.sig_el;
    case CH_EXC: {
        if (eps <= E_EXC) return 0.0;
        double x = eps / E_EXC;
        return c.sig_x0 * std::log(x) / x;
    }
    case CH_IZ:
        if (eps <= E_ION) return 0.0;
        return c.lotz_a * 2.0 * std::log(eps / E_ION) / (eps * E_ION);
    case CH_CX: return c.sig_cx;
    case CH_IEL: return c.sig_iel;
    }
    return 0.0;
}

// Null-collision bound: max of n_g sigma_T(eps(g)) g on a dense grid of relative
// speeds up to the largest expected one, with a 0.1 % margin.
double numax_of(const pic_config &c, bool ion, double m, double sig_n)
{
    if (!(c.ng > 0.0)) return 0.0;
    double mu = m * MASS_HE / (m + MASS_HE);
    double ecap = ion ? std::fabs(c.V) + 40.0 * c.Ti0 : std::fabs(c.V) + 40.0 * c.Te0 + 40.0 * c.Tc;
    double gcap = std::sqrt(2.0 * Q_E * ecap / m) + 6.0 * sig_n;
    double best = 0.0;
    for (int i = 1; i <= 65536; ++i) {
        double g = gcap * (double)i / 65536.0;
        double eps = 0.5 * mu * g * g / Q_E;
        double sig = ion ? sigma_ch(c, CH_CX, eps) + sigma_ch(c, CH_IEL, eps)
                         : sigma_ch(c, CH_EEL, eps) + sigma_ch(c, CH_EXC, eps) + sigma_ch(c, CH_IZ, eps);
        double nu = c.ng * sig * g;
        if (nu > best) best = nu;
    }
    return best * 1.001;
}

int check_cfg(const pic_config &c)
{
    if (c.N < 2 || c.N > 32767) return fail(PIC_EINVAL, "N must be in [2, 32767]");
    if (!(c.L > 0.0) || !(c.dt > 0.0)) return fail(PIC_EINVAL, "L and dt must be positive");
    if (c.n_load < 1 || c.n_load > (1ll << 29)) return fail(PIC_EINVAL, "n_load must be in [1, 2^29]");
    if (c.ng < 0.0 || c.gamma_emit < 0.0 || c.Te0 < 0.0 || c.Ti0 < 0.0 || c.Tc < 0.0 || c.Tne < 0.0 ||
        c.Tni < 0.0 || c.n0 < 0.0)
        return fail(PIC_EINVAL, "negative density, flux or temperature");
    if (c.tally_period < 1) return fail(PIC_EINVAL, "tally_period must be >= 1");
    if (c.flags != 0) return fail(PIC_EINVAL, "flags must be 0");
    return PIC_OK;
}

void derive(const pic_config &c, pic_derived &d)
{
    d.dz = c.L / (double)c.N;
    d.invdz = (double)c.N / c.L;
    d.w0 = c.n0 * c.L / (double)c.n_load;
    double mi = MASS_HE - MASS_E;
    double sne = std::sqrt(Q_E * c.Tne / MASS_HE), sni = std::sqrt(Q_E * c.Tni / MASS_HE);
    d.numax[0] = numax_of(c, false, MASS_E, sne);
    d.numax[1] = numax_of(c, true, mi, sni);
    d.lam[0] = d.numax[0] * c.dt;
    d.lam[1] = d.numax[1] * c.dt;
    d.emit_per_step = d.w0 > 0.0 ? c.gamma_emit * c.dt / d.w0 : 0.0;
    double f = c.capacity_factor > 0.0 ? c.capacity_factor : 1.6;
    int64_t cap = (int64_t)std::ceil(f * (double)c.n_load) + 4096;
    cap = (cap + 2047) / 2048 * 2048;   // a multiple of the largest particle chunk
    for (int s = 0; s < NSP; ++s) d.capacity[s] = cap;
}

// ----------------------------------------------------------------------------
// Workspace layout: one bump allocation per array, 256-byte aligned.
// ----------------------------------------------------------------------------
struct Bump {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        off = (off + ALIGN - 1) / ALIGN * ALIGN;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

void layout(const pic_config *cfgs, int nd, const std::vector<pic_derived> &der, Bump &bp,
            std::vector<Diode> &hD, Diode *&dD, long long *&dNload, size_t &zero_end)
{
    dD = bp.take<Diode>(nd);
    dNload = bp.take<long long>(nd);
    // everything below is cleared at init
    size_t zero_begin = bp.off;
    (void)zero_begin;
    DiodeState *st = bp.take<DiodeState>(nd);
    DiodeTally *tl = bp.take<DiodeTally>(nd);
    hD.assign(nd, Diode{});
    for (int d = 0; d < nd; ++d) {
        Diode &D = hD[d];
        const int nn = cfgs[d].N + 1;
        D.st = st ? st + d : nullptr;
        D.tally = tl ? tl + d : nullptr;
        D.ring = bp.take<TallySnap>(RING);
        D.izq = bp.take<IzEvent>(IZQ_CAP);
        for (int s = 0; s < NSP; ++s) {
            D.H[s] = bp.take<unsigned long long>(nn);
            D.Hlast[s] = bp.take<long long>(nn);
            D.Hsum[s] = bp.take<long long>(nn);
            D.cell_cnt[s] = bp.take<int32_t>(nn);
        }
        D.phi = bp.take<double>(nn);
        D.E = bp.take<double>(nn);
        D.phi_sum = bp.take<double>(nn);
        D.agg = bp.take<FieldAgg>((nn + FIELD_BIG_TILE - 1) / FIELD_BIG_TILE);     // one per large-grid tile
        D.agg_flag = bp.take<uint32_t>((nn + FIELD_BIG_TILE - 1) / FIELD_BIG_TILE);
        D.tacc = bp.take<TallyCopy>(TALLY_COPIES);
    }
    zero_end = bp.off;
    for (int d = 0; d < nd; ++d) {
        Diode &D = hD[d];
        for (int p = 0; p < 2; ++p)
            for (int s = 0; s < NSP; ++s) {
                size_t cap = (size_t)der[d].capacity[s];
                D.buf[p][s].z = bp.take<double>(cap);
                D.buf[p][s].vz = bp.take<float>(cap);
                D.buf[p][s].tc = bp.take<uint32_t>(cap);
                D.buf[p][s].cold = bp.take<ColdRec>(cap);
            }
        for (int s = 0; s < NSP; ++s) D.rare[s] = bp.take<uint32_t>((size_t)der[d].capacity[s]);
    }
}

void fill_params(const pic_config &c, const pic_derived &der, Diode &D)
{
    D.L = c.L;
    D.dz = der.dz;
    D.invdz = der.invdz;
    D.V = c.V;
    D.dt = c.dt;
    D.w0 = der.w0;
    D.alpha = Q_E * der.w0 * der.dz / (4294967296.0 * EPS0);
    D.N = c.N;
    for (int s = 0; s < NSP; ++s) D.cap[s] = (int32_t)der.capacity[s];
    const double mi = MASS_HE - MASS_E;
    D.mass[SP_P] = D.mass[SP_E] = MASS_E;
    D.mass[SP_I] = mi;
    D.qmdt[SP_P] = D.qmdt[SP_E] = -Q_E / MASS_E * c.dt;
    D.qmdt[SP_I] = Q_E / mi * c.dt;
    for (int ion = 0; ion < 2; ++ion) {
        const double m = ion ? mi : MASS_E;
        const double mu = m * MASS_HE / (m + MASS_HE);
        D.numax[ion] = der.numax[ion];
        D.lam[ion] = der.lam[ion];
        D.numax_f[ion] = (float)der.numax[ion];
        D.sig_n[ion] = (float)std::sqrt(Q_E * (ion ? c.Tni : c.Tne) / MASS_HE);
        D.half_mu_over_e[ion] = (float)(0.5 * mu / Q_E);
        D.mfrac_m[ion] = (float)(m / (m + MASS_HE));
        D.mfrac_M[ion] = (float)(MASS_HE / (m + MASS_HE));
        D.two_e_over_mu[ion] = (float)(2.0 * Q_E / mu);
    }
    D.ng = (float)c.ng;
    D.sig_el = (float)c.sig_el;
    D.sig_x0 = (float)c.sig_x0;
    D.lotz_a2 = (float)(2.0 * c.lotz_a / E_ION);
    D.sig_cx = (float)c.sig_cx;
    D.sig_iel = (float)c.sig_iel;
    D.emit_x = der.emit_per_step;
    D.sig_c = std::sqrt(Q_E * c.Tc / MASS_E);
    D.sig_e0 = std::sqrt(Q_E * c.Te0 / MASS_E);
    D.sig_i0 = std::sqrt(Q_E * c.Ti0 / mi);
    // a state-loaded particle starts inside the energy range the null-collision
    // bound was scanned over (numax_of)
    D.load_cap_ev[0] = std::fabs(c.V) + 40.0 * c.Te0 + 40.0 * c.Tc;
    D.load_cap_ev[1] = std::fabs(c.V) + 40.0 * c.Ti0;
    D.kseed = c.seed ^ c.diode;
    D.channels = c.channels;
    D.replenish = c.replenish;
    D.tally_period = c.tally_period;
}

}  // namespace

// A captured run of steps: an optional re-sort, then r steps (particle kernel
// and sources / field kernels each).  Timed variants carry event-record
// nodes around some of the particle kernels.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipGraph_t src = nullptr;             // timed: kept alive, its node handles address the exec's nodes
    std::vector<hipGraphNode_t> marks;    // timed: (start, end) event nodes per timed step
    uint64_t last_use = 0;
};

struct pic_handle {
    int nd = 0;
    std::vector<pic_config> cfg;
    std::vector<pic_derived> der;
    char *ws = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    std::vector<Diode> hD;
    Diode *dD = nullptr;
    long long *dNload = nullptr;
    DiodeState *dS = nullptr;   // state array (diode d at dS + d)
    int max_nodes = 0;
    int64_t issued = 0;         // steps enqueued so far (re-sort schedule)
    int parity = 0;             // current particle buffer (flips with every re-sort)
    bool sort_next = true;      // force a re-sort before the next step
    int ppt = 2;
    int grid = 1024;
    int sort_period = 64;
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;   // private stream used only for graph capture
    // captured runs keyed by (parity, re-sort first, timed, steps); the least
    // recently used is dropped beyond GRAPH_CACHE entries
    std::map<int64_t, GraphEntry> graphs;
    uint64_t use_clock = 0;
    std::vector<hipEvent_t> evpool;         // pic_step_timed's events, created on demand, reused
    hipEvent_t tev[2] = {nullptr, nullptr}; // placeholders for event nodes not timed in a replay
    hipEvent_t tt[2] = {nullptr, nullptr};  // start and end of a timed run
    void drop_graphs()
    {
        for (auto &kv : graphs) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            if (kv.second.src) (void)hipGraphDestroy(kv.second.src);
        }
        graphs.clear();
    }
    ~pic_handle()
    {
        drop_graphs();
        for (auto e : evpool) (void)hipEventDestroy(e);
        for (auto e : tev)
            if (e) (void)hipEventDestroy(e);
        for (auto e : tt)
            if (e) (void)hipEventDestroy(e);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
    std::vector<std::array<int64_t, NSP>> live_offset;
};

namespace {

int grid_for(const pic_handle *h)
{
    int64_t chunks = 0;
    for (int d = 0; d < h->nd; ++d)
        for (int s = 0; s < NSP; ++s) chunks += (h->der[d].capacity[s] + 256 * h->ppt - 1) / (256 * h->ppt);
    int64_t g = std::min<int64_t>(chunks, 8192);
    g = std::max<int64_t>(8, (g + 7) / 8 * 8);
    return (int)g;
}

// parity: buffer current before the re-sort; the re-sort flips it
int enqueue_sort(pic_handle *h, hipStream_t s, int parity)
{
    HIP_TRY(picx_launch_sort(h->dD, h->dS, h->nd, h->ppt, h->grid, parity, s));
    return PIC_OK;
}

int enqueue_body(pic_handle *h, hipStream_t s, int parity)
{
    HIP_TRY(picx_launch_particles(h->dD, h->dS, h->nd, 0, h->ppt, h->grid, parity, s));
    HIP_TRY(picx_launch_sources_field(h->dD, h->dS, h->nd, 0, h->max_nodes, parity, s));
    return PIC_OK;
}

bool sort_due(const pic_handle *h)
{
    return h->sort_next || (h->sort_period > 0 && h->issued % h->sort_period == 0);
}

int launch_step(pic_handle *h)
{
    if (sort_due(h)) {
        int rc = enqueue_sort(h, h->stream, h->parity);
        if (rc) return rc;
        h->parity ^= 1;
        h->sort_next = false;
    }
    int rc = enqueue_body(h, h->stream, h->parity);
    if (rc) return rc;
    h->issued++;
    return PIC_OK;
}

// Steps from the current schedule position to the next re-sort boundary (at
// most `left`): the run one graph replays.
int64_t run_length(const pic_handle *h, int64_t left)
{
    int64_t r = left;
    if (h->sort_period > 0) r = std::min<int64_t>(r, h->sort_period - h->issued % h->sort_period);
    return std::max<int64_t>(r, 1);
}

// Schedule bookkeeping after a run of r steps that began with a re-sort or not.
void advance(pic_handle *h, bool sorted, int64_t r)
{
    if (sorted) {
        h->parity ^= 1;
        h->sort_next = false;
    }
    h->issued += r;
}

// Splice event-record nodes around ns particle kernels spread evenly over the
// r steps of a captured chain (optional re-sort kernels, then per step the
// particle kernel and the sources / field kernels).
int splice_timing(pic_handle *h, hipGraph_t g, int r, std::vector<hipGraphNode_t> &marks)
{
    size_t nn = 0;
    if (hipGraphGetNodes(g, nullptr, &nn) != hipSuccess) return fail(PIC_EHIP, "hipGraphGetNodes failed");
    std::vector<hipGraphNode_t> nodes(nn), chain;
    if (hipGraphGetNodes(g, nodes.data(), &nn) != hipSuccess) return fail(PIC_EHIP, "hipGraphGetNodes failed");
    hipGraphNode_t cur = nullptr;
    for (auto nd : nodes) {
        size_t nd_in = 0;
        if (hipGraphNodeGetDependencies(nd, nullptr, &nd_in) != hipSuccess)
            return fail(PIC_EHIP, "dependency query failed");
        if (nd_in == 0) {
            if (cur) return fail(PIC_EHIP, "captured run is not a chain");
            cur = nd;
        }
    }
    while (cur) {
        chain.push_back(cur);
        size_t nout = 0;
        if (hipGraphNodeGetDependentNodes(cur, nullptr, &nout) != hipSuccess || nout > 1)
            return fail(PIC_EHIP, "captured run is not a chain");
        hipGraphNode_t next = nullptr;
        if (nout == 1 && hipGraphNodeGetDependentNodes(cur, &next, &nout) != hipSuccess)
            return fail(PIC_EHIP, "dependency query failed");
        cur = nout ? next : nullptr;
    }
    const int B = 1 + picx_sources_field_kernels(h->max_nodes, 0);   // kernels per step
    if ((int)chain.size() < B * r) return fail(PIC_EHIP, "unexpected captured run");
    const int first = (int)chain.size() - B * r;      // particle kernel of the run's first step
    const int ns = std::min(TPOS, r);
    marks.assign(2 * ns, nullptr);
    for (int j = 0; j < ns; ++j) {
        const int k = (int)((int64_t)j * r / ns);
        const int at = first + B * k;
        hipGraphNode_t part = chain[at], field = chain[at + 1];
        hipGraphNode_t pred = at > 0 ? chain[at - 1] : nullptr;
        const size_t npred = pred ? 1 : 0;
        if ((pred && hipGraphRemoveDependencies(g, &pred, &part, 1) != hipSuccess) ||
            hipGraphRemoveDependencies(g, &part, &field, 1) != hipSuccess ||
            hipGraphAddEventRecordNode(&marks[2 * j], g, pred ? &pred : nullptr, npred, h->tev[0]) != hipSuccess ||
            hipGraphAddDependencies(g, &marks[2 * j], &part, 1) != hipSuccess ||
            hipGraphAddEventRecordNode(&marks[2 * j + 1], g, &part, 1, h->tev[1]) != hipSuccess ||
            hipGraphAddDependencies(g, &marks[2 * j + 1], &field, 1) != hipSuccess)
            return fail(PIC_EHIP, "splicing event nodes failed");
    }
    return PIC_OK;
}

// The captured run (parity p, re-sort first or not, r steps, timed or not),
// captured and instantiated on first use.
int get_graph(pic_handle *h, int p, bool sorted, int64_t r, bool timed, GraphEntry **out)
{
    const int64_t key = (int64_t)p | (int64_t)sorted << 1 | (int64_t)timed << 2 | r << 3;
    auto it = h->graphs.find(key);
    if (it != h->graphs.end()) {
        it->second.last_use = ++h->use_clock;
        *out = &it->second;
        return PIC_OK;
    }
    if (h->graphs.size() >= GRAPH_CACHE) {
        // drop the least recently used; nothing of it may still be in flight
        HIP_TRY(hipStreamSynchronize(h->stream));
        auto lru = h->graphs.begin();
        for (auto q = h->graphs.begin(); q != h->graphs.end(); ++q)
            if (q->second.last_use < lru->second.last_use) lru = q;
        if (lru->second.exec) (void)hipGraphExecDestroy(lru->second.exec);
        if (lru->second.src) (void)hipGraphDestroy(lru->second.src);
        h->graphs.erase(lru);
    }
    if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    // timing placeholders of the captured event nodes (see pic_step_timed)
    for (auto &e : h->tev)
        if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    hipGraph_t g;
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = sorted ? enqueue_sort(h, h->cap_stream, p) : PIC_OK;
    const int q = sorted ? p ^ 1 : p;
    for (int64_t k = 0; rc == PIC_OK && k < r; ++k) rc = enqueue_body(h, h->cap_stream, q);
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (rc) return rc;
    if (e != hipSuccess) return fail(PIC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    GraphEntry ent;
    if (timed && (rc = splice_timing(h, g, (int)r, ent.marks))) {
        (void)hipGraphDestroy(g);
        return rc;
    }
    e = hipGraphInstantiate(&ent.exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(PIC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    if (timed) ent.src = g;     // the exec's event nodes are addressed through it
    else (void)hipGraphDestroy(g);
    ent.last_use = ++h->use_clock;
    *out = &(h->graphs[key] = ent);
    return PIC_OK;
}

// Enqueue nsteps steps.  With graph replay each run up to the next re-sort
// boundary is one graph launch (whole re-sort periods once the schedule is
// aligned); otherwise every step is launched on the stream.
int run_steps(pic_handle *h, int64_t nsteps)
{
    int64_t left = nsteps;
    while (left > 0) {
        if (!h->use_graph) {
            int rc = launch_step(h);
            if (rc) return rc;
            --left;
            continue;
        }
        const bool sorted = sort_due(h);
        const int64_t r = run_length(h, left);
        GraphEntry *g;
        int rc = get_graph(h, h->parity, sorted, r, false, &g);
        if (rc) return rc;
        HIP_TRY(hipGraphLaunch(g->exec, h->stream));
        advance(h, sorted, r);
        left -= r;
    }
    return PIC_OK;
}

int refield(pic_handle *h)
{
    HIP_TRY(picx_launch_sort(h->dD, h->dS, h->nd, h->ppt, h->grid, h->parity, h->stream));
    h->parity ^= 1;
    HIP_TRY(picx_launch_particles(h->dD, h->dS, h->nd, 1, h->ppt, h->grid, h->parity, h->stream));
    HIP_TRY(picx_launch_sources_field(h->dD, h->dS, h->nd, 1, h->max_nodes, h->parity, h->stream));
    h->sort_next = false;
    return PIC_OK;
}

int read_state(pic_handle *h, int d, DiodeState &st, DiodeTally &t)
{
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpy(&st, h->hD[d].st, sizeof(st), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&t, h->hD[d].tally, sizeof(t), hipMemcpyDeviceToHost));
    return PIC_OK;
}

void live_counts(const pic_handle *h, int d, const DiodeTally &t, int64_t out[NSP])
{
    const int64_t nl = h->cfg[d].n_load;
    int64_t born[NSP] = {nl + (int64_t)t.n_iz + (int64_t)t.n_repl, (int64_t)t.n_emit,
                         nl + (int64_t)t.n_iz + (int64_t)t.n_repl};
    for (int s = 0; s < NSP; ++s)
        out[s] = born[s] - (int64_t)t.abs_count[s][0] - (int64_t)t.abs_count[s][1] + h->live_offset[d][s];
}

int err_code(uint32_t bits)
{
    if (bits & ERR_CAPACITY) return fail(PIC_ENOSPACE, "particle capacity exceeded on the device");
    if (bits & ERR_NULLCOLL) return fail(PIC_ENULLCOLL, "collision frequency exceeded the null-collision bound");
    if (bits & ERR_IZQ) return fail(PIC_ERANGE, "ionisation queue overflow");
    if (bits & ERR_RANGE)
        return fail(PIC_ERANGE, "a node's deposit reached 2^53 (2^21 particles of one species on one node)");
    if (bits & ERR_NAN) return fail(PIC_ENAN, "non-finite particle position");
    return PIC_OK;
}

// Boundary diagnostics over a window of tallies ("Benchmark cases": Gamma_net,
// backflow ratio, efficiencies; "Boundary energy diagnostics": eqs. 1-10).
void diag_window(const pic_config &c, double w0, double window_s, const DiodeTally &a, const DiodeTally &b,
                 pic_diag &o)
{
    const double inv = w0 / window_s;
    for (int s = 0; s < NSP; ++s)
        for (int w = 0; w < 2; ++w) {
            o.gamma_abs[s][w] = (double)(b.abs_count[s][w] - a.abs_count[s][w]) * inv;
            o.q_abs[s][w] = (b.abs_energy[s][w] - a.abs_energy[s][w]) * inv;
        }
    const double ge = c.gamma_emit;
    o.gamma_emit = ge;
    o.gamma_emit_meas = (double)(b.n_emit - a.n_emit) * inv;
    o.gamma_ref = o.gamma_abs[SP_E][0];
    o.gamma_anode = o.gamma_abs[SP_E][1];
    o.gamma_net = ge - o.gamma_ref;
    o.backflow_pct = ge > 0.0 ? 100.0 * o.gamma_ref / ge : NAN;
    o.eta_net = ge > 0.0 ? o.gamma_net / ge : NAN;
    o.eta_anode = ge > 0.0 ? o.gamma_anode / ge : NAN;
    const double kbe = K_B / Q_E;
    const double AR = 1.20e6 / (kbe * kbe);          // A m^-2 eV^-2
    const double Tc = c.Tc;
    o.wf_eff = (ge > 0.0 && Tc > 0.0) ? -Tc * std::log(Q_E * ge / (AR * Tc * Tc)) : NAN;
    o.q_emit_theory = ge * Q_E * (o.wf_eff + 2.0 * Tc);
    o.q_ion_cath_recomb = o.gamma_abs[SP_I][0] * Q_E * E_ION;
    o.q_cool1 = o.q_emit_theory - o.q_abs[SP_E][0] - o.q_abs[SP_P][0] - o.q_abs[SP_I][0];
    o.q_cool2 = o.q_cool1 - o.q_ion_cath_recomb;
    o.q_anode1 = o.q_abs[SP_E][1] + o.q_abs[SP_P][1] + o.q_abs[SP_I][1];
    o.q_ion_anode_recomb = o.gamma_abs[SP_I][1] * Q_E * E_ION;
    o.q_anode2 = o.q_anode1 + o.q_ion_anode_recomb;
    o.phi_vc_eff = (ge > 0.0 && o.gamma_net > 0.0) ? Tc * std::log(o.gamma_net / ge) : NAN;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char *pic_last_error(void) { return g_err.c_str(); }

int pic_derive(const pic_config *cfg, pic_derived *out)
{
    if (!cfg || !out) return fail(PIC_EINVAL, "null argument");
    int rc = check_cfg(*cfg);
    if (rc) return rc;
    derive(*cfg, *out);
    return PIC_OK;
}

int pic_workspace_size(const pic_config *cfgs, int n_diodes, size_t *bytes)
{
    if (!cfgs || !bytes || n_diodes < 1 || n_diodes > PIC_MAX_DIODES) return fail(PIC_EINVAL, "bad arguments");
    std::vector<pic_derived> der(n_diodes);
    for (int d = 0; d < n_diodes; ++d) {
        int rc = check_cfg(cfgs[d]);
        if (rc) return rc;
        derive(cfgs[d], der[d]);
    }
    Bump bp{nullptr};
    std::vector<Diode> hD;
    Diode *dD;
    long long *dN;
    size_t zend;
    layout(cfgs, n_diodes, der, bp, hD, dD, dN, zend);
    *bytes = (bp.off + ALIGN - 1) / ALIGN * ALIGN;
    return PIC_OK;
}

// dens == nullptr: uniform load; else the warm-start loader over dens
// [n_diodes][2][max N] (device).
// dens: null for the uniform load, else [n_diodes][rows][max N] with rows 2
// (densities) or PIC_STATE_ROWS (densities, potential, velocity quantiles)
static int init_impl(const pic_config *cfgs, int n_diodes, void *dev_workspace, size_t bytes, void *hip_stream,
                     const double *dens, int rows, pic_handle **out)
{
    if (!cfgs || !out || !dev_workspace || n_diodes < 1 || n_diodes > PIC_MAX_DIODES)
        return fail(PIC_EINVAL, "bad arguments");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % ALIGN) return fail(PIC_EINVAL, "workspace not 256-byte aligned");
    size_t need;
    int rc = pic_workspace_size(cfgs, n_diodes, &need);
    if (rc) return rc;
    if (bytes < need) return fail(PIC_ENOSPACE, "workspace too small");
    pic_handle *h = new (std::nothrow) pic_handle;
    if (!h) return fail(PIC_ENOSPACE, "host allocation failed");
    h->nd = n_diodes;
    h->cfg.assign(cfgs, cfgs + n_diodes);
    h->der.resize(n_diodes);
    for (int d = 0; d < n_diodes; ++d) derive(cfgs[d], h->der[d]);
    h->ws = static_cast<char *>(dev_workspace);
    h->bytes = bytes;
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->live_offset.assign(n_diodes, std::array<int64_t, NSP>{0, 0, 0});
    h->sort_period = cfgs[0].sort_period > 0 ? cfgs[0].sort_period : 64;
    Bump bp{h->ws};
    size_t zend;
    layout(cfgs, n_diodes, h->der, bp, h->hD, h->dD, h->dNload, zend);
    for (int d = 0; d < n_diodes; ++d) {
        fill_params(cfgs[d], h->der[d], h->hD[d]);
        h->max_nodes = std::max(h->max_nodes, cfgs[d].N + 1);
    }
    h->dS = h->hD[0].st;
    h->grid = grid_for(h);

    auto cleanup = [&](int code) { delete h; return code; };
    if (picx_prepare() != hipSuccess) return cleanup(fail(PIC_EHIP, "kernel attribute setup failed"));
    size_t zbeg = (reinterpret_cast<char *>(h->hD[0].st) - h->ws);
    if (hipMemsetAsync(h->ws + zbeg, 0, zend - zbeg, h->stream) != hipSuccess)
        return cleanup(fail(PIC_EHIP, "hipMemsetAsync failed"));
    std::vector<DiodeState> st(n_diodes);
    std::vector<long long> nl(n_diodes);
    long long maxl = 0;
    for (int d = 0; d < n_diodes; ++d) {
        std::memset(&st[d], 0, sizeof(DiodeState));
        st[d].n[SP_P] = st[d].n[SP_I] = (int32_t)cfgs[d].n_load;
        st[d].next_id = (uint32_t)(2 * cfgs[d].n_load);
        nl[d] = cfgs[d].n_load;
        maxl = std::max(maxl, nl[d]);
    }
    if (hipMemcpyAsync(h->dD, h->hD.data(), sizeof(Diode) * n_diodes, hipMemcpyHostToDevice, h->stream) ||
        hipMemcpyAsync(h->dNload, nl.data(), sizeof(long long) * n_diodes, hipMemcpyHostToDevice, h->stream) ||
        hipMemcpyAsync(h->hD[0].st, st.data(), sizeof(DiodeState) * n_diodes, hipMemcpyHostToDevice, h->stream))
        return cleanup(fail(PIC_EHIP, "hipMemcpyAsync failed"));
    if (!dens) {
        if (picx_launch_load(h->dD, h->dNload, n_diodes, maxl, h->stream) != hipSuccess)
            return cleanup(fail(PIC_EHIP, "load launch failed"));
    } else {
        int max_cells = 0;
        for (int d = 0; d < n_diodes; ++d) max_cells = std::max(max_cells, cfgs[d].N);
        if (picx_launch_profile_load(h->dD, dens, rows, n_diodes, max_cells, h->stream) != hipSuccess)
            return cleanup(fail(PIC_EHIP, "profile load launch failed"));
    }
    // the staging vectors die here: wait for the copies
    if (hipStreamSynchronize(h->stream) != hipSuccess) return cleanup(fail(PIC_EHIP, "sync failed"));
    if (dens) {
        for (int d = 0; d < n_diodes; ++d) {
            DiodeState sd;
            if (hipMemcpy(&sd, h->hD[d].st, sizeof(sd), hipMemcpyDeviceToHost) != hipSuccess)
                return cleanup(fail(PIC_EHIP, "state read failed"));
            const uint32_t err = sd.err;
            // live counts are births minus losses from n_load: offset by what was loaded
            h->live_offset[d][SP_P] = (int64_t)sd.n[SP_P] - cfgs[d].n_load;
            h->live_offset[d][SP_I] = (int64_t)sd.n[SP_I] - cfgs[d].n_load;
            if (err & ERR_NAN)
                return cleanup(fail(PIC_ENAN, "diode " + std::to_string(d) +
                                                  ": density profile negative, not finite or above 2^30 per cell, "
                                                  "or a state entry not finite"));
            if (err & ERR_CAPACITY)
                return cleanup(fail(PIC_ENOSPACE, "diode " + std::to_string(d) +
                                                      ": profile holds more particles than the capacity "
                                                      "(raise capacity_factor or n_load)"));
        }
    }
    rc = refield(h);
    if (rc) return cleanup(rc);
    *out = h;
    return PIC_OK;
}

int pic_init(const pic_config *cfgs, int n_diodes, void *dev_workspace, size_t bytes, void *hip_stream,
             pic_handle **out)
{
    return init_impl(cfgs, n_diodes, dev_workspace, bytes, hip_stream, nullptr, 0, out);
}

int pic_init_from_profiles(const pic_config *cfgs, int n_diodes, void *dev_workspace, size_t bytes,
                           void *hip_stream, const double *dev_dens, pic_handle **out)
{
    if (!dev_dens) return fail(PIC_EINVAL, "null density profiles");
    return init_impl(cfgs, n_diodes, dev_workspace, bytes, hip_stream, dev_dens, 2, out);
}

static_assert(PIC_STATE_ROWS == STATE_ROWS, "state layout of the ABI and the kernels");

int pic_init_from_state(const pic_config *cfgs, int n_diodes, void *dev_workspace, size_t bytes, void *hip_stream,
                        const double *dev_state, pic_handle **out)
{
    if (!dev_state) return fail(PIC_EINVAL, "null state");
    return init_impl(cfgs, n_diodes, dev_workspace, bytes, hip_stream, dev_state, PIC_STATE_ROWS, out);
}

int pic_step(pic_handle *h, int64_t nsteps)
{
    if (!h || nsteps < 0) return fail(PIC_EINVAL, "bad arguments");
    return run_steps(h, nsteps);
}

int pic_sync(pic_handle *h)
{
    if (!h) return fail(PIC_EINVAL, "null handle");
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int d = 0; d < h->nd; ++d) {
        uint32_t err = 0;
        HIP_TRY(hipMemcpy(&err, &h->hD[d].st->err, sizeof(err), hipMemcpyDeviceToHost));
        if (err) return err_code(err);
    }
    return PIC_OK;
}

static void fill_tally(const pic_handle *h, int diode, const DiodeTally &t, pic_tally *out)
{
    std::memset(out, 0, sizeof(*out));
    live_counts(h, diode, t, out->n_live);
    for (int s = 0; s < NSP; ++s)
        for (int w = 0; w < 2; ++w) {
            out->abs_count[s][w] = (int64_t)t.abs_count[s][w];
            out->abs_energy[s][w] = t.abs_energy[s][w];
        }
    out->n_emit = (int64_t)t.n_emit;
    out->n_repl = (int64_t)t.n_repl;
    out->n_iz = (int64_t)t.n_iz;
    for (int k = 0; k < 2; ++k) out->cand[k] = (int64_t)t.cand[k];
    for (int k = 0; k < NCH; ++k) out->coll[k] = (int64_t)t.coll[k];
    out->rare_spill = (int64_t)t.rare_spill;
    out->resorts = (int64_t)t.resorts;
    out->resorts_ions_kept = (int64_t)t.resorts_ions_kept;
}

int pic_get_snapshot(pic_handle *h, int diode, int64_t step, pic_tally *out)
{
    if (!h || !out || diode < 0 || diode >= h->nd || step < 0) return fail(PIC_EINVAL, "bad arguments");
    const int64_t D = h->cfg[diode].tally_period;
    if (step % D) return fail(PIC_EINVAL, "step must be a multiple of tally_period");
    DiodeState st;
    DiodeTally now;
    int rc = read_state(h, diode, st, now);
    if (rc) return rc;
    if (step > (int64_t)st.step) return fail(PIC_EINVAL, "step not reached yet");
    DiodeTally t;
    std::memset(&t, 0, sizeof(t));
    if (step > 0) {
        TallySnap sn;
        HIP_TRY(hipMemcpy(&sn, h->hD[diode].ring + (step / D) % RING, sizeof(sn), hipMemcpyDeviceToHost));
        if ((int64_t)sn.step != step) return fail(PIC_ERANGE, "snapshot no longer in the ring");
        t = sn.t;
    }
    fill_tally(h, diode, t, out);
    out->step = step;
    out->err_bits = st.err;
    return PIC_OK;
}

int pic_get_tally(pic_handle *h, int diode, pic_tally *out)
{
    if (!h || !out || diode < 0 || diode >= h->nd) return fail(PIC_EINVAL, "bad arguments");
    DiodeState st;
    DiodeTally t;
    int rc = read_state(h, diode, st, t);
    if (rc) return rc;
    fill_tally(h, diode, t, out);
    out->step = st.step;
    out->next_id = st.next_id;
    out->err_bits = st.err;
    return PIC_OK;
}

int pic_diagnostics(pic_handle *h, int diode, int64_t window_steps, pic_diag *out)
{
    if (!h || !out || diode < 0 || diode >= h->nd || window_steps < 0) return fail(PIC_EINVAL, "bad arguments");
    const pic_config &c = h->cfg[diode];
    DiodeState st;
    DiodeTally now;
    int rc = read_state(h, diode, st, now);
    if (rc) return rc;
    std::memset(out, 0, sizeof(*out));
    DiodeTally zero;
    std::memset(&zero, 0, sizeof(zero));
    const int64_t D = c.tally_period;
    int64_t e_step = st.step, b_step = 0;
    DiodeTally tb = zero, te = now;
    if (window_steps > 0) {
        if (window_steps % D) return fail(PIC_EINVAL, "window_steps must be a multiple of tally_period");
        e_step = (int64_t)st.step / D * D;
        b_step = e_step - window_steps;
        if (b_step < 0) return fail(PIC_EINVAL, "window reaches before step 0");
        if (window_steps / D >= RING) return fail(PIC_EINVAL, "window longer than the snapshot ring");
        auto snap_at = [&](int64_t s, DiodeTally &t) -> int {
            if (s == 0) { t = zero; return PIC_OK; }
            TallySnap sn;
            HIP_TRY(hipMemcpy(&sn, h->hD[diode].ring + (s / D) % RING, sizeof(sn), hipMemcpyDeviceToHost));
            if ((int64_t)sn.step != s) return fail(PIC_ERANGE, "snapshot no longer in the ring");
            t = sn.t;
            return PIC_OK;
        };
        if ((rc = snap_at(b_step, tb))) return rc;
        if ((rc = snap_at(e_step, te))) return rc;
    }
    if (e_step <= b_step) return fail(PIC_EINVAL, "empty window");
    out->step_begin = b_step;
    out->step_end = e_step;
    diag_window(c, h->der[diode].w0, (double)(e_step - b_step) * c.dt, tb, te, *out);
    int64_t live[NSP];
    live_counts(h, diode, te, live);
    for (int s = 0; s < NSP; ++s) out->n_live[s] = (double)live[s];
    return err_code(st.err);
}

int pic_avg_reset(pic_handle *h, int on) { return pic_avg_control(h, -1, on); }

int pic_avg_control(pic_handle *h, int diode, int on)
{
    if (!h || diode < -1 || diode >= h->nd) return fail(PIC_EINVAL, "bad arguments");
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int d = 0; d < h->nd; ++d) {
        if (diode >= 0 && d != diode) continue;
        const Diode &D = h->hD[d];
        const size_t nn = h->cfg[d].N + 1;
        for (int s = 0; s < NSP; ++s) HIP_TRY(hipMemsetAsync(D.Hsum[s], 0, nn * sizeof(long long), h->stream));
        HIP_TRY(hipMemsetAsync(D.phi_sum, 0, nn * sizeof(double), h->stream));
        int v[2] = {on ? 1 : 0, 0};
        HIP_TRY(hipMemcpyAsync(&D.st->avg_on, v, sizeof(v), hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipMemsetAsync(&D.st->phi_slope_sum, 0, sizeof(double), h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    return PIC_OK;
}

int pic_get_fields(pic_handle *h, int diode, double *phi, double *n_e, double *n_i, int time_avg)
{
    if (!h || diode < 0 || diode >= h->nd) return fail(PIC_EINVAL, "bad arguments");
    HIP_TRY(hipStreamSynchronize(h->stream));
    const Diode &D = h->hD[diode];
    const int nn = h->cfg[diode].N + 1;
    DiodeState st;
    HIP_TRY(hipMemcpy(&st, D.st, sizeof(st), hipMemcpyDeviceToHost));
    const double navg = time_avg ? (double)std::max(st.avg_steps, 1) : 1.0;
    if (time_avg && st.avg_steps == 0) return fail(PIC_EINVAL, "no time average accumulated");
    if (phi) {
        // the large-grid field step stores phi less phi_slope j (zero on smaller grids)
        HIP_TRY(hipMemcpy(phi, time_avg ? D.phi_sum : D.phi, nn * sizeof(double), hipMemcpyDeviceToHost));
        const double slope = time_avg ? st.phi_slope_sum : st.phi_slope;
        for (int j = 0; j < nn; ++j) phi[j] = (phi[j] + slope * (double)j) / navg;
    }
    std::vector<long long> H[NSP];
    for (int s = 0; s < NSP; ++s) {
        H[s].resize(nn);
        HIP_TRY(hipMemcpy(H[s].data(), time_avg ? D.Hsum[s] : D.Hlast[s], nn * sizeof(long long),
                          hipMemcpyDeviceToHost));
    }
    const double k = h->der[diode].w0 / (4294967296.0 * h->der[diode].dz * navg);
    for (int j = 0; j < nn; ++j) {
        const double vol = (j == 0 || j == nn - 1) ? 2.0 : 1.0;
        if (n_e) n_e[j] = k * vol * ((double)H[SP_P][j] + (double)H[SP_E][j]);
        if (n_i) n_i[j] = k * vol * (double)H[SP_I][j];
    }
    return PIC_OK;
}

int pic_get_hist(pic_handle *h, int diode, int species, int64_t *out)
{
    if (!h || !out || diode < 0 || diode >= h->nd || species < 0 || species >= NSP)
        return fail(PIC_EINVAL, "bad arguments");
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipMemcpy(out, h->hD[diode].Hlast[species], (h->cfg[diode].N + 1) * sizeof(int64_t),
                      hipMemcpyDeviceToHost));
    return PIC_OK;
}

static_assert(PIC_PHASE_MAX_BINS == PHASE_MAX_BINS, "phase-space bin limit");

// p is device memory on the GPU that holds ref (the handle's workspace).
static bool device_memory_beside(const void *p, const void *ref)
{
    hipPointerAttribute_t a{}, b{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess || hipPointerGetAttributes(&b, ref) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice && a.device == b.device;
}

int pic_phase_space(pic_handle *h, int diode, int species, int nz, int nv, double vmin, double vmax,
                    uint64_t *dev_out)
{
    if (!h || !dev_out || diode < 0 || diode >= h->nd || species < 0 || species >= NSP)
        return fail(PIC_EINVAL, "bad arguments");
    if (nz < 1 || nv < 1 || (int64_t)nz * (nv + 2) > PIC_PHASE_MAX_BINS)
        return fail(PIC_EINVAL, "need nz >= 1, nv >= 1 and nz * (nv + 2) <= PIC_PHASE_MAX_BINS");
    if (!std::isfinite(vmin) || !std::isfinite(vmax) || !(vmax > vmin))
        return fail(PIC_EINVAL, "need finite vmin < vmax");
    if (!device_memory_beside(dev_out, h->ws))
        return fail(PIC_EINVAL, "dev_out must be device memory on the handle's GPU");
    const double sz = (double)nz / h->cfg[diode].L;
    const double sv = (double)nv / (vmax - vmin);
    const int64_t cap = h->der[diode].capacity[species];
    const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (cap + 4095) / 4096));
    HIP_TRY(picx_launch_phase_hist(h->dD, h->dS, diode, species, h->parity, nz, nv, sz, vmin, sv,
                                   reinterpret_cast<unsigned long long *>(dev_out), blocks, h->stream));
    return PIC_OK;
}

int pic_get_efield(pic_handle *h, int diode, double *out)
{
    if (!h || !out || diode < 0 || diode >= h->nd) return fail(PIC_EINVAL, "bad arguments");
    HIP_TRY(hipStreamSynchronize(h->stream));
    const int nn = h->cfg[diode].N + 1;
    DiodeState st;
    HIP_TRY(hipMemcpy(&st, h->hD[diode].st, sizeof(st), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(out, h->hD[diode].E, nn * sizeof(double), hipMemcpyDeviceToHost));
    // the large-grid field step stores E less a uniform shift (zero on smaller grids)
    for (int j = 0; j < nn; ++j) out[j] += st.e_shift;
    return PIC_OK;
}

int pic_get_particles(pic_handle *h, int diode, int species, int64_t cap, int64_t *n_out, double *z, float *vx,
                      float *vy, float *vz, uint32_t *id, uint32_t *tc)
{
    if (!h || !n_out || diode < 0 || diode >= h->nd || species < 0 || species >= NSP || cap < 0)
        return fail(PIC_EINVAL, "bad arguments");
    DiodeState st;
    DiodeTally t;
    int rc = read_state(h, diode, st, t);
    if (rc) return rc;
    const int n = st.n[species];
    const SpeciesBuf &b = h->hD[diode].buf[st.parity ^ st.flip[species]][species];
    std::vector<double> hz(n);
    std::vector<float> hvz(n);
    std::vector<uint32_t> htc(n);
    std::vector<ColdRec> hcold(n);
    if (n > 0) {
        HIP_TRY(hipMemcpy(hz.data(), b.z, n * sizeof(double), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(hvz.data(), b.vz, n * sizeof(float), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(htc.data(), b.tc, n * sizeof(uint32_t), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(hcold.data(), b.cold, n * sizeof(ColdRec), hipMemcpyDeviceToHost));
    }
    std::vector<int> idx;
    idx.reserve(n);
    for (int i = 0; i < n; ++i)
        if (hz[i] >= 0.0) idx.push_back(i);
    std::sort(idx.begin(), idx.end(), [&](int a, int c) { return hcold[a].id < hcold[c].id; });
    *n_out = (int64_t)idx.size();
    if ((int64_t)idx.size() > cap) return fail(PIC_ENOSPACE, "output capacity too small");
    for (size_t k = 0; k < idx.size(); ++k) {
        const int i = idx[k];
        if (z) z[k] = hz[i];
        if (vx) vx[k] = hcold[i].vx;
        if (vy) vy[k] = hcold[i].vy;
        if (vz) vz[k] = hvz[i];
        if (id) id[k] = hcold[i].id;
        if (tc) tc[k] = htc[i];
    }
    return PIC_OK;
}

int pic_set_particles(pic_handle *h, int diode, int species, int64_t n, const double *z, const float *vx,
                      const float *vy, const float *vz, const uint32_t *id, const uint32_t *tc)
{
    if (!h || diode < 0 || diode >= h->nd || species < 0 || species >= NSP || n < 0)
        return fail(PIC_EINVAL, "bad arguments");
    if (n > 0 && (!z || !vx || !vy || !vz || !id || !tc)) return fail(PIC_EINVAL, "null array");
    if (n > h->der[diode].capacity[species]) return fail(PIC_ENOSPACE, "more particles than capacity");
    for (int64_t i = 0; i < n; ++i) {
        if (!(z[i] > 0.0 && z[i] < h->cfg[diode].L)) return fail(PIC_EINVAL, "particle outside (0, L)");
        if (!std::isfinite(vx[i]) || !std::isfinite(vy[i]) || !std::isfinite(vz[i]))
            return fail(PIC_ENAN, "non-finite particle velocity");
    }
    DiodeState st;
    DiodeTally t;
    int rc = read_state(h, diode, st, t);
    if (rc) return rc;
    const SpeciesBuf &b = h->hD[diode].buf[st.parity ^ st.flip[species]][species];
    if (n > 0) {
        std::vector<ColdRec> hcold(n);
        for (int64_t i = 0; i < n; ++i) hcold[i] = ColdRec{vx[i], vy[i], id[i], 0u};
        HIP_TRY(hipMemcpy(b.z, z, n * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(b.vz, vz, n * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(b.tc, tc, n * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(b.cold, hcold.data(), n * sizeof(ColdRec), hipMemcpyHostToDevice));
    }
    // the slots are unsorted: all of them are the tail (n_new = 0), which the
    // next re-sort sorts
    const int32_t nn = (int32_t)n, zero = 0;
    HIP_TRY(hipMemcpy(&h->hD[diode].st->n[species], &nn, sizeof(nn), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(&h->hD[diode].st->n_new[species], &zero, sizeof(zero), hipMemcpyHostToDevice));
    int64_t live[NSP];
    live_counts(h, diode, t, live);
    h->live_offset[diode][species] += n - live[species];
    h->sort_next = true;
    return PIC_OK;
}

int pic_set_counters(pic_handle *h, int diode, int64_t step, uint32_t next_id)
{
    if (!h || diode < 0 || diode >= h->nd || step < 0 || step >= 0xFFFFFFFFll) return fail(PIC_EINVAL, "bad arguments");
    HIP_TRY(hipStreamSynchronize(h->stream));
    uint32_t v[2] = {next_id, (uint32_t)step};
    static_assert(offsetof(DiodeState, step) == offsetof(DiodeState, next_id) + 4, "layout");
    HIP_TRY(hipMemcpy(&h->hD[diode].st->next_id, v, sizeof(v), hipMemcpyHostToDevice));
    // the record block's flag holds the step it last finished + 1: cleared, it
    // cannot match a step the counters were moved back to
    const uint32_t zero = 0u;
    HIP_TRY(hipMemcpy(&h->hD[diode].st->rec_flag, &zero, sizeof(zero), hipMemcpyHostToDevice));
    return PIC_OK;
}

int pic_refield(pic_handle *h)
{
    if (!h) return fail(PIC_EINVAL, "null handle");
    return refield(h);
}

int pic_step_timed(pic_handle *h, int64_t nsteps, double *particle_kernel_ms, double *total_ms)
{
    if (!h || nsteps < 1) return fail(PIC_EINVAL, "bad arguments");
    // events: up to TPOS particle kernels per replayed graph, or one launch in
    // `every` on the plain stream, at most TIMED_MAX kernels in all.  On the
    // plain stream each timestamp pair stalls the launches around it, so few
    // kernels are sampled there (at most PLAIN_SAMPLES; four on short runs),
    // with an odd stride: the samples fall on every position of a re-sort
    // period (whose length is a power of two), not on the same few.
    const int64_t want = std::min<int64_t>(PLAIN_SAMPLES, std::max<int64_t>(4, nsteps / 16));
    const int64_t every = nsteps <= want ? 1 : ((nsteps + want - 1) / want) | 1;
    auto pair = [&](int64_t k, hipEvent_t &a, hipEvent_t &b) -> int {
        while ((int64_t)h->evpool.size() < 2 * (k + 1)) {
            // timing only: their timestamps are read once the run's end
            // event (with the default fence) has synchronised; without a
            // system-scope fence the record does not write back and
            // invalidate the caches around the kernel it brackets
            hipEvent_t e;
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
            h->evpool.push_back(e);
        }
        a = h->evpool[2 * k];
        b = h->evpool[2 * k + 1];
        return PIC_OK;
    };
    for (auto &e : h->tt)
        if (!e) HIP_TRY(hipEventCreate(&e));
    int rc;
    HIP_TRY(hipEventRecord(h->tt[0], h->stream));
    int64_t k_ev = 0, left = nsteps, k = 0;
    while (left > 0) {
        const bool sorted = sort_due(h);
        if (h->use_graph) {
            const int64_t r = run_length(h, left);
            GraphEntry *g;
            if ((rc = get_graph(h, h->parity, sorted, r, true, &g))) return rc;
            // every event node of the replay gets a fresh pooled event, or a
            // placeholder once TIMED_MAX kernels are timed
            for (size_t j = 0; j + 1 < g->marks.size(); j += 2) {
                hipEvent_t a = h->tev[0], b = h->tev[1];
                if (k_ev < TIMED_MAX) {
                    if ((rc = pair(k_ev, a, b))) return rc;
                    ++k_ev;
                }
                HIP_TRY(hipGraphExecEventRecordNodeSetEvent(g->exec, g->marks[j], a));
                HIP_TRY(hipGraphExecEventRecordNodeSetEvent(g->exec, g->marks[j + 1], b));
            }
            HIP_TRY(hipGraphLaunch(g->exec, h->stream));
            advance(h, sorted, r);
            left -= r;
            k += r;
            continue;
        }
        if (sorted) {
            if ((rc = enqueue_sort(h, h->stream, h->parity))) return rc;
            h->parity ^= 1;
            h->sort_next = false;
        }
        hipEvent_t a = nullptr, b = nullptr;
        const bool rec = (k % every) == 0 && k_ev < TIMED_MAX;
        if (rec) {
            if ((rc = pair(k_ev, a, b))) return rc;
            ++k_ev;
            HIP_TRY(hipEventRecord(a, h->stream));
        }
        HIP_TRY(picx_launch_particles(h->dD, h->dS, h->nd, 0, h->ppt, h->grid, h->parity, h->stream));
        if (rec) HIP_TRY(hipEventRecord(b, h->stream));
        HIP_TRY(picx_launch_sources_field(h->dD, h->dS, h->nd, 0, h->max_nodes, h->parity, h->stream));
        h->issued++;
        --left;
        ++k;
    }
    HIP_TRY(hipEventRecord(h->tt[1], h->stream));
    HIP_TRY(hipEventSynchronize(h->tt[1]));
    double acc = 0.0;
    for (int64_t q = 0; q < k_ev; ++q) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->evpool[2 * q], h->evpool[2 * q + 1]));
        acc += ms;
    }
    float tot = 0.f;
    HIP_TRY(hipEventElapsedTime(&tot, h->tt[0], h->tt[1]));
    if (k_ev == 0) return fail(PIC_EHIP, "no particle kernel was timed");
    if (particle_kernel_ms) *particle_kernel_ms = acc / (double)k_ev;
    if (total_ms) *total_ms = tot;
    return PIC_OK;
}

int pic_set_tuning(pic_handle *h, int ppt, int grid, int sort_period, int use_graph)
{
    if (!h) return fail(PIC_EINVAL, "null handle");
    if (ppt != 0 && ppt != 1 && ppt != 2 && ppt != 4 && ppt != 8) return fail(PIC_EINVAL, "ppt must be 1, 2, 4 or 8");
    if (grid < 0 || grid > 65536 || sort_period < 0) return fail(PIC_EINVAL, "bad grid or sort period");
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (ppt) h->ppt = ppt;
    h->grid = grid ? (grid + 7) / 8 * 8 : grid_for(h);
    if (sort_period) h->sort_period = sort_period;
    if (use_graph >= 0) h->use_graph = use_graph != 0;
    h->drop_graphs();
    return PIC_OK;
}

int pic_get_tuning(pic_handle *h, int *ppt, int *grid, int *sort_period, int *use_graph)
{
    if (!h) return fail(PIC_EINVAL, "null handle");
    if (ppt) *ppt = h->ppt;
    if (grid) *grid = h->grid;
    if (sort_period) *sort_period = h->sort_period;
    if (use_graph) *use_graph = h->use_graph ? 1 : 0;
    return PIC_OK;
}

// Launch-schedule autotuner: a full search over particles per thread, re-sort
// period and grid size, the best four re-timed, then graph replay, each
// candidate timed with HIP events over whole re-sort periods of real steps
// (the diodes advance).
int pic_autotune(pic_handle *h, int64_t trial_steps, int *ppt, int *grid, int *sort_period, int *use_graph,
                 double *ms_per_step)
{
    if (!h || trial_steps < 1) return fail(PIC_EINVAL, "bad arguments");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto timed = [&](int p, int g, int k, int ug, double &ms) -> int {
        int rc = pic_set_tuning(h, p, g, k, ug);
        if (rc) return rc;
        // align to a re-sort boundary and warm the new schedule: one period,
        // or two with graph replay, whose graphs are captured per buffer
        // parity and the re-sort flips it every period (a capture inside the
        // timed steps would count against replay)
        int64_t pad = (h->sort_period - h->issued % h->sort_period) % h->sort_period;
        if ((rc = run_steps(h, pad + (ug ? 2 : 1) * h->sort_period))) return rc;
        const int64_t n = std::max<int64_t>(1, (trial_steps + h->sort_period - 1) / h->sort_period) * h->sort_period;
        HIP_TRY(hipEventRecord(e0, h->stream));
        if ((rc = run_steps(h, n))) return rc;
        HIP_TRY(hipEventRecord(e1, h->stream));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        ms = t / (double)n;
        return PIC_OK;
    };
    int bp = h->ppt, bk = h->sort_period, bu = h->use_graph ? 1 : 0;
    int bg = h->grid;
    double best = 1e300, ms;
    int rc;
    // full search over particles per thread, re-sort period and grid (the
    // coordinate-wise search stalled in local optima)
    struct Cand {
        int p, k, g;
        double sum;
        int n;
    };
    std::vector<Cand> cands;
    // besides the listed grids, the one that gives each block eight chunks of
    // the particles the stores hold now (eight chunks per block measured best
    // where that grid falls between two listed ones)
    std::vector<int64_t> slots;
    for (int d = 0; d < h->nd; ++d) {
        DiodeState st;
        DiodeTally t;
        if ((rc = read_state(h, d, st, t))) return rc;
        for (int s = 0; s < NSP; ++s) slots.push_back(st.n[s]);
    }
    for (int p : {1, 2, 4}) {
        int64_t chunks = 0;
        for (int64_t n : slots) chunks += (n + 256 * p - 1) / (256 * p);
        const int g8 = (int)std::min<int64_t>(65536, std::max<int64_t>(256, (chunks + 7) / 8));
        // powers of two and the points half way between them (the best grid
        // is not monotone in the chunks per block: the paper's eleven-flux
        // batch ran 71.9 us per step at 3072 blocks, 73.0 at 4096)
        std::vector<int> grids = {2048, 3072, 4096, 6144, 8192, 12288, 16384};
        bool near = false;
        for (int g : grids) near = near || std::abs(g - g8) * 10 < g;
        if (!near) grids.push_back(g8);
        for (int k : {16, 32, 64, 128})
            for (int g : grids) {
                if ((rc = timed(p, g, k, bu, ms))) return rc;
                cands.push_back(Cand{p, k, h->grid, ms, 1});
            }
    }
    // the best few again, twice each and interleaved (the run drifts between
    // trials, and one trial's noise is a few per cent, as large as the
    // differences between the best schedules): the lowest mean wins
    std::stable_sort(cands.begin(), cands.end(), [](const Cand &x, const Cand &y) { return x.sum < y.sum; });
    const size_t top = std::min<size_t>(4, cands.size());
    for (int r = 0; r < 2; ++r)
        for (size_t c = 0; c < top; ++c) {
            if ((rc = timed(cands[c].p, cands[c].g, cands[c].k, bu, ms))) return rc;
            cands[c].sum += ms;
            cands[c].n += 1;
        }
    for (size_t c = 0; c < top; ++c) {
        const double mean = cands[c].sum / cands[c].n;
        if (mean < best) {
            best = mean;
            bp = cands[c].p;
            bk = cands[c].k;
            bg = cands[c].g;
        }
    }
    // then graph replay on or off: three trials each, alternating, lowest mean
    double sum[2] = {0.0, 0.0};
    for (int r = 0; r < 3; ++r)
        for (int u : {0, 1}) {
            if ((rc = timed(bp, bg, bk, u, ms))) return rc;
            sum[u] += ms;
        }
    bu = sum[1] < sum[0] ? 1 : 0;
    best = sum[bu] / 3.0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if ((rc = pic_set_tuning(h, bp, bg, bk, bu))) return rc;
    if (ppt) *ppt = bp;
    if (grid) *grid = h->grid;
    if (sort_period) *sort_period = bk;
    if (use_graph) *use_graph = bu;
    if (ms_per_step) *ms_per_step = best;
    return PIC_OK;
}

int pic_steady_from_series(const double *br, const double *n_live, int nblocks, double tol_pp, double tol_rel,
                           int *steady_block, double *br_steady, int *n_mean)
{
    if (!br || !n_live || nblocks < 0 || !steady_block || !br_steady || !n_mean || !(tol_pp > 0.0) ||
        !(tol_rel > 0.0))
        return fail(PIC_EINVAL, "bad arguments");
    *steady_block = -1;
    *br_steady = NAN;
    *n_mean = 0;
    for (int b = 2; b < nblocks; ++b) {
        const bool br_ok = std::fabs(br[b] - br[b - 1]) < tol_pp && std::fabs(br[b] - br[b - 2]) < tol_pp;
        const bool n_ok = n_live[b] > 0.0 && std::fabs(n_live[b] - n_live[b - 1]) / n_live[b] < tol_rel;
        if (br_ok && n_ok) {
            *steady_block = b;
            double acc = 0.0;
            int m = 0;
            for (int q = b + 1; q < nblocks && q <= b + 4; ++q, ++m) acc += br[q];
            *n_mean = m;
            *br_steady = m ? acc / m : NAN;
            return PIC_OK;
        }
    }
    return PIC_OK;
}

int pic_steady_state(pic_handle *h, int diode, int block_tallies, double tol_pp, double tol_rel, pic_steady *out)
{
    if (!h || !out || diode < 0 || diode >= h->nd || block_tallies < 1) return fail(PIC_EINVAL, "bad arguments");
    const pic_config &c = h->cfg[diode];
    DiodeState st;
    DiodeTally now;
    int rc = read_state(h, diode, st, now);
    if (rc) return rc;
    std::vector<TallySnap> ring(RING);
    HIP_TRY(hipMemcpy(ring.data(), h->hD[diode].ring, sizeof(TallySnap) * RING, hipMemcpyDeviceToHost));
    const int64_t D = c.tally_period, blk = D * block_tallies;
    const int64_t last = (int64_t)st.step / blk;     // complete blocks
    const int64_t first = std::max<int64_t>(0, last - (RING / block_tallies) + 1);
    auto snap = [&](int64_t stepno, DiodeTally &t) -> bool {
        if (stepno == 0) { std::memset(&t, 0, sizeof(t)); return true; }
        const TallySnap &sn = ring[(stepno / D) % RING];
        if ((int64_t)sn.step != stepno) return false;
        t = sn.t;
        return true;
    };
    std::vector<double> br, nl;
    int64_t b0 = -1;
    for (int64_t b = first; b < last; ++b) {
        DiodeTally ta, tb;
        if (!snap(b * blk, ta) || !snap((b + 1) * blk, tb)) { br.clear(); nl.clear(); b0 = -1; continue; }
        if (b0 < 0) b0 = b;
        const double win = (double)blk * c.dt;
        const double g_ref = (double)(tb.abs_count[SP_E][0] - ta.abs_count[SP_E][0]) * h->der[diode].w0 / win;
        br.push_back(c.gamma_emit > 0.0 ? 100.0 * g_ref / c.gamma_emit : 0.0);
        int64_t live[NSP];
        live_counts(h, diode, tb, live);
        nl.push_back((double)(live[0] + live[1] + live[2]));
    }
    std::memset(out, 0, sizeof(*out));
    out->blocks = (int)br.size();
    out->block_steps = blk;
    int sb = -1, nm = 0;
    double bs = NAN;
    if ((rc = pic_steady_from_series(br.data(), nl.data(), (int)br.size(), tol_pp, tol_rel, &sb, &bs, &nm)))
        return rc;
    out->steady = sb >= 0 ? 1 : 0;
    out->steady_step = sb >= 0 ? (b0 + sb + 1) * blk : -1;
    out->backflow_pct = bs;
    out->blocks_averaged = nm;
    out->last_backflow_pct = br.empty() ? NAN : br.back();
    return PIC_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Checkpoint: a self-describing host image of every diode's state at a step
// boundary.  Layout: header {magic, version, n_diodes, bytes}, then per diode
// its configuration, state block, tallies, snapshot ring, live-count offsets,
// node arrays (H, last H, H sums, phi, E, phi sum) and per species the slot
// count and the slots (z, v_z, t_c, {v_x, v_y, id}) of the current buffer.
// ----------------------------------------------------------------------------
namespace {

constexpr char CKPT_MAGIC[8] = {'P', 'I', 'C', 'C', 'K', 'P', 'T', '1'};
constexpr uint32_t CKPT_VERSION = 4;

struct CkptHeader {
    char magic[8];
    uint32_t version;
    int32_t nd;
    uint64_t bytes;
};

bool same_physics(const pic_config &a, const pic_config &b)
{
    return a.L == b.L && a.N == b.N && a.V == b.V && a.n0 == b.n0 && a.Te0 == b.Te0 && a.Ti0 == b.Ti0 &&
           a.n_load == b.n_load && a.gamma_emit == b.gamma_emit && a.Tc == b.Tc && a.ng == b.ng &&
           a.Tne == b.Tne && a.Tni == b.Tni && a.dt == b.dt && a.sig_el == b.sig_el && a.sig_x0 == b.sig_x0 &&
           a.lotz_a == b.lotz_a && a.sig_cx == b.sig_cx && a.sig_iel == b.sig_iel && a.channels == b.channels &&
           a.replenish == b.replenish && a.seed == b.seed && a.diode == b.diode &&
           a.tally_period == b.tally_period;
}

size_t ckpt_bytes(const pic_handle *h, const std::vector<DiodeState> &st)
{
    size_t b = sizeof(CkptHeader);
    for (int d = 0; d < h->nd; ++d) {
        const size_t nn = (size_t)h->cfg[d].N + 1;
        b += sizeof(pic_config) + sizeof(DiodeState) + sizeof(DiodeTally) + sizeof(TallySnap) * RING +
             sizeof(int64_t) * NSP;
        b += nn * (3 * 3 * sizeof(int64_t) + 3 * sizeof(double));
        for (int s = 0; s < NSP; ++s)
            b += sizeof(int32_t) + (size_t)st[d].n[s] * (sizeof(double) + sizeof(float) + sizeof(uint32_t) +
                                                          sizeof(ColdRec));
    }
    return b;
}

int read_states(pic_handle *h, std::vector<DiodeState> &st)
{
    HIP_TRY(hipStreamSynchronize(h->stream));
    st.resize(h->nd);
    HIP_TRY(hipMemcpy(st.data(), h->hD[0].st, sizeof(DiodeState) * h->nd, hipMemcpyDeviceToHost));
    return PIC_OK;
}

// device <-> host copy of one region, advancing the host cursor
template <bool SAVE>
int xfer(char *&cur, void *dev, size_t n)
{
    if (n == 0) return PIC_OK;
    if (SAVE) HIP_TRY(hipMemcpy(cur, dev, n, hipMemcpyDeviceToHost));
    else HIP_TRY(hipMemcpy(dev, cur, n, hipMemcpyHostToDevice));
    cur += n;
    return PIC_OK;
}

}  // namespace

extern "C" {

int pic_checkpoint_size(pic_handle *h, size_t *bytes)
{
    if (!h || !bytes) return fail(PIC_EINVAL, "bad arguments");
    std::vector<DiodeState> st;
    int rc = read_states(h, st);
    if (rc) return rc;
    *bytes = ckpt_bytes(h, st);
    return PIC_OK;
}

int pic_save(pic_handle *h, void *host_buf, size_t bytes, size_t *written)
{
    if (!h || !host_buf) return fail(PIC_EINVAL, "bad arguments");
    std::vector<DiodeState> st;
    int rc = read_states(h, st);
    if (rc) return rc;
    const size_t need = ckpt_bytes(h, st);
    if (bytes < need) return fail(PIC_ENOSPACE, "checkpoint buffer too small (pic_checkpoint_size)");
    char *cur = static_cast<char *>(host_buf);
    CkptHeader hd;
    std::memcpy(hd.magic, CKPT_MAGIC, 8);
    hd.version = CKPT_VERSION;
    hd.nd = h->nd;
    hd.bytes = need;
    std::memcpy(cur, &hd, sizeof(hd));
    cur += sizeof(hd);
    for (int d = 0; d < h->nd; ++d) {
        const Diode &D = h->hD[d];
        const size_t nn = (size_t)h->cfg[d].N + 1;
        std::memcpy(cur, &h->cfg[d], sizeof(pic_config));
        cur += sizeof(pic_config);
        std::memcpy(cur, &st[d], sizeof(DiodeState));
        cur += sizeof(DiodeState);
        if ((rc = xfer<true>(cur, D.tally, sizeof(DiodeTally))) || (rc = xfer<true>(cur, D.ring, sizeof(TallySnap) * RING)))
            return rc;
        std::memcpy(cur, h->live_offset[d].data(), sizeof(int64_t) * NSP);
        cur += sizeof(int64_t) * NSP;
        for (int s = 0; s < NSP; ++s)
            if ((rc = xfer<true>(cur, D.H[s], nn * 8)) || (rc = xfer<true>(cur, D.Hlast[s], nn * 8)) ||
                (rc = xfer<true>(cur, D.Hsum[s], nn * 8)))
                return rc;
        if ((rc = xfer<true>(cur, D.phi, nn * 8)) || (rc = xfer<true>(cur, D.E, nn * 8)) ||
            (rc = xfer<true>(cur, D.phi_sum, nn * 8)))
            return rc;
        for (int s = 0; s < NSP; ++s) {
            const SpeciesBuf &b = D.buf[st[d].parity ^ st[d].flip[s]][s];
            const int32_t n = st[d].n[s];
            std::memcpy(cur, &n, sizeof(n));
            cur += sizeof(n);
            if ((rc = xfer<true>(cur, b.z, (size_t)n * 8)) || (rc = xfer<true>(cur, b.vz, (size_t)n * 4)) ||
                (rc = xfer<true>(cur, b.tc, (size_t)n * 4)) || (rc = xfer<true>(cur, b.cold, (size_t)n * sizeof(ColdRec))))
                return rc;
        }
    }
    if (written) *written = need;
    return PIC_OK;
}

int pic_load(pic_handle *h, const void *host_buf, size_t bytes)
{
    if (!h || !host_buf || bytes < sizeof(CkptHeader)) return fail(PIC_EINVAL, "bad arguments");
    CkptHeader hd;
    std::memcpy(&hd, host_buf, sizeof(hd));
    if (std::memcmp(hd.magic, CKPT_MAGIC, 8) != 0 || hd.version != CKPT_VERSION)
        return fail(PIC_EINVAL, "not a checkpoint of this library version");
    if (hd.nd != h->nd) return fail(PIC_EINVAL, "checkpoint holds a different number of diodes");
    if (hd.bytes > bytes) return fail(PIC_EINVAL, "checkpoint truncated");
    // validate every diode before touching the device
    const char *cur = static_cast<const char *>(host_buf) + sizeof(hd);
    const char *end = static_cast<const char *>(host_buf) + hd.bytes;
    std::vector<DiodeState> st(h->nd);
    {
        const char *c = cur;
        for (int d = 0; d < h->nd; ++d) {
            pic_config cfg;
            if (c + sizeof(pic_config) + sizeof(DiodeState) > end) return fail(PIC_EINVAL, "checkpoint truncated");
            std::memcpy(&cfg, c, sizeof(cfg));
            if (!same_physics(cfg, h->cfg[d])) return fail(PIC_EINVAL, "checkpoint of a different configuration");
            c += sizeof(pic_config);
            std::memcpy(&st[d], c, sizeof(DiodeState));
            c += sizeof(DiodeState) + sizeof(DiodeTally) + sizeof(TallySnap) * RING + sizeof(int64_t) * NSP;
            const size_t nn = (size_t)cfg.N + 1;
            c += nn * (3 * 3 * 8 + 3 * 8);
            for (int s = 0; s < NSP; ++s) {
                int32_t n;
                if (c + sizeof(n) > end) return fail(PIC_EINVAL, "checkpoint truncated");
                std::memcpy(&n, c, sizeof(n));
                if (n < 0 || n > h->der[d].capacity[s] || n != st[d].n[s])
                    return fail(PIC_ENOSPACE, "checkpoint particles exceed this handle's capacity");
                c += sizeof(n);
                if (c + (size_t)n * (8 + 4 + 4 + sizeof(ColdRec)) > end) return fail(PIC_EINVAL, "checkpoint truncated");
                // slots hold live particles (0 < z < L) or holes (z < 0); velocities finite
                const char *zc = c, *vc = c + (size_t)n * 8, *cc0 = c + (size_t)n * 16;
                for (int32_t i = 0; i < n; ++i) {
                    double z;
                    float vz;
                    ColdRec cr;
                    std::memcpy(&z, zc + (size_t)i * 8, 8);
                    std::memcpy(&vz, vc + (size_t)i * 4, 4);
                    std::memcpy(&cr, cc0 + (size_t)i * sizeof(ColdRec), sizeof(ColdRec));
                    if (!std::isfinite(z) || !std::isfinite(vz) || !std::isfinite(cr.vx) || !std::isfinite(cr.vy))
                        return fail(PIC_ENAN, "checkpoint holds a non-finite particle");
                    if (z >= cfg.L || z == 0.0) return fail(PIC_EINVAL, "checkpoint particle outside the gap");
                }
                c += (size_t)n * (8 + 4 + 4 + sizeof(ColdRec));
            }
            if (c > end) return fail(PIC_EINVAL, "checkpoint truncated");
        }
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    char *cc = const_cast<char *>(cur);
    int rc;
    for (int d = 0; d < h->nd; ++d) {
        const Diode &D = h->hD[d];
        const size_t nn = (size_t)h->cfg[d].N + 1;
        cc += sizeof(pic_config);
        DiodeState s0 = st[d];
        s0.parity = h->parity;   // the slots go into this handle's current buffer
        for (int s = 0; s < NSP; ++s) {
            s0.flip[s] = 0;
            s0.keep[s] = 0;
        }
        s0.arrive = 0;           // no field step is in flight at a step boundary
        s0.spill_flag = 0u;
        s0.field_epoch = 0u;     // with the tile flags cleared below
        cc += sizeof(DiodeState);
        if ((rc = xfer<false>(cc, D.tally, sizeof(DiodeTally))) || (rc = xfer<false>(cc, D.ring, sizeof(TallySnap) * RING)))
            return rc;
        std::memcpy(h->live_offset[d].data(), cc, sizeof(int64_t) * NSP);
        cc += sizeof(int64_t) * NSP;
        for (int s = 0; s < NSP; ++s)
            if ((rc = xfer<false>(cc, D.H[s], nn * 8)) || (rc = xfer<false>(cc, D.Hlast[s], nn * 8)) ||
                (rc = xfer<false>(cc, D.Hsum[s], nn * 8)))
                return rc;
        if ((rc = xfer<false>(cc, D.phi, nn * 8)) || (rc = xfer<false>(cc, D.E, nn * 8)) ||
            (rc = xfer<false>(cc, D.phi_sum, nn * 8)))
            return rc;
        for (int s = 0; s < NSP; ++s) {
            const SpeciesBuf &b = D.buf[h->parity][s];
            int32_t n;
            std::memcpy(&n, cc, sizeof(n));
            cc += sizeof(n);
            if ((rc = xfer<false>(cc, b.z, (size_t)n * 8)) || (rc = xfer<false>(cc, b.vz, (size_t)n * 4)) ||
                (rc = xfer<false>(cc, b.tc, (size_t)n * 4)) ||
                (rc = xfer<false>(cc, b.cold, (size_t)n * sizeof(ColdRec))))
                return rc;
        }
        HIP_TRY(hipMemcpy(D.st, &s0, sizeof(DiodeState), hipMemcpyHostToDevice));
        // per-step scratch starts clear
        for (int s = 0; s < NSP; ++s) HIP_TRY(hipMemset(D.cell_cnt[s], 0, nn * sizeof(int32_t)));
        HIP_TRY(hipMemset(D.tacc, 0, sizeof(TallyCopy) * TALLY_COPIES));
        HIP_TRY(hipMemset(D.agg_flag, 0, sizeof(uint32_t) * ((nn + FIELD_BIG_TILE - 1) / FIELD_BIG_TILE)));
    }
    h->sort_next = true;
    return PIC_OK;
}

}  // extern "C"

extern "C" {

void pic_destroy(pic_handle *h) { delete h; }

}  // extern "C"
