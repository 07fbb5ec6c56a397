// pic_kernels.hip -- gfx950 kernels of the 1D3V PIC-MCC thermionic diode.
//
// One step of every diode is two launches (plus a cell re-sort every K
// steps):
//   k_particles       gather (LDS field tile) -> leapfrog push -> electrode
//                     absorption -> null-collision MCC (compacted candidate
//                     queue) -> 64-bit fixed-point CIC deposit into an LDS
//                     window histogram flushed with global integer atomics;
//   k_field_step /    one block per node tile of every diode plus one for
//   k_field_tiles     the newborn records: ionisation products (ordered by
//                     parent id), thermionic emission, pair replenishment,
//                     then the exact-integer double prefix-scan Poisson solve
//                     and the field, tallies and snapshots (k_field_tiles on
//                     grids above 2049 nodes).
// Particles are processed in chunks of 256*PPT slots; the chunk list spans all
// (diode, species) segments.  Each block of the particle kernel takes an equal
// share of it, in an order that puts every segment's unsorted tail (the
// particles born since the last re-sort) before the sorted bodies.
#include "pic_internal.h"

namespace pic {

constexpr int NT = 256;            // threads per particle block
constexpr int NW = NT / 64;        // wavefronts per particle block
constexpr int WMAX = 512;          // LDS window (nodes) of the field tile / histogram
constexpr int QW_SLACK = 384;      // per-wave LDS queue of rare items: 64 PPT + QW_SLACK entries
constexpr int DRIFT = 160;         // cells of drift since the last re-sort kept in the LDS window
constexpr int BIN_SHIFT = 5;       // the re-sort orders particles by bins of 32 cells
// The re-sort counts bins in LDS (up to WMAX + 1 of them: every bin of grids
// up to 16416 cells).  On larger grids a run's window is its first and last
// bin with this margin, wide enough for the fastest electrons of a period (a
// particle outside takes a global counter atomic and four partial-line
// stores of its own).
constexpr int SORT_DRIFT_B = 64;

__host__ __device__ constexpr int nbins_of(int N) { return ((N - 1) >> BIN_SHIFT) + 1; }
// The counter / offset of bin b lives at cell slot b << BIN_SHIFT of the count
// array: 128 bytes apart, so that the device-scope atomics of many blocks on
// the bins spread over memory channels instead of queueing on one.
__device__ __forceinline__ int bin_slot(int b) { return b << BIN_SHIFT; }

// Device views of the particle and grid arrays in the global address space.
// Pointers loaded from the Diode block are generic, and generic accesses
// compile to flat_* instructions, which count in the LDS counter as well as
// the vector-memory one: every wait for an LDS result would then also wait
// for all flat loads and stores in flight, the next chunk's prefetch
// included.  global_* instructions count only in the vector-memory counter.
#define GLB __attribute__((address_space(1)))
struct GBuf {
    GLB double *z;
    GLB float *vz;
    GLB uint32_t *tc;
    GLB ColdRec *cold;
};
__device__ __forceinline__ GBuf gbuf(const SpeciesBuf &b)
{
    return GBuf{(GLB double *)b.z, (GLB float *)b.vz, (GLB uint32_t *)b.tc, (GLB ColdRec *)b.cold};
}
template <class T>
__device__ __forceinline__ GLB T *glb(T *p)
{
    return (GLB T *)p;
}
__device__ __forceinline__ void gadd(GLB unsigned long long *p, unsigned long long v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int gadd(GLB int *p, int v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Cold records move as one 16-byte vector (a struct cannot be assigned in
// another address space).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ ColdRec get_cold(const GLB ColdRec *p)
{
    const u32x4 v = *(const GLB u32x4 *)p;
    return ColdRec{__uint_as_float(v.x), __uint_as_float(v.y), v.z, v.w};
}
__device__ __forceinline__ void put_cold(GLB ColdRec *p, float vx, float vy, uint32_t id)
{
    *(GLB u32x4 *)p = u32x4{__float_as_uint(vx), __float_as_uint(vy), id, 0u};
}
constexpr int FT = 1024;           // threads of the sources / field blocks
constexpr int FW = FT / 64;
constexpr double TWO32 = 4294967296.0;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32 -> 64-bit
// multiplies, Weyl key schedule.  Keyed by (particle id, seed ^ diode),
// counter (step, event, sub, 0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Uniforms: all exactly representable, strictly inside (0, 1).
__device__ __forceinline__ float u24f(uint32_t w)
{
    return (float)((w >> 9) * 2u + 1u) * 5.9604644775390625e-8f;
}
__device__ __forceinline__ double u32d(uint32_t w) { return ((double)w + 0.5) * 2.3283064365386963e-10; }
__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo)
{
    unsigned long long m = ((unsigned long long)hi << 20) | (unsigned long long)(lo >> 12);
    return ((double)m * 2.0 + 1.0) * 1.1102230246251565e-16;
}

// Box-Muller in FP32 on 24-bit uniforms (collision draws).
__device__ __forceinline__ void bm24(uint32_t a, uint32_t b, float &n1, float &n2)
{
    float r = sqrtf(-2.0f * logf(u24f(a)));
    float s, c;
    sincospif(2.0f * u24f(b), &s, &c);
    n1 = r * c;
    n2 = r * s;
}
// Box-Muller in FP64 on 32-bit uniforms (loads and births).
__device__ __forceinline__ void bm32(uint32_t a, uint32_t b, double &n1, double &n2)
{
    double r = sqrt(-2.0 * log(u32d(a)));
    double s, c;
    sincospi(2.0 * u32d(b), &s, &c);
    n1 = r * c;
    n2 = r * s;
}

// Step at which a particle is next a null-collision candidate: the free flight
// of a rate-numax Poisson process, -ln(U)/numax, rounded up to whole steps.
__device__ __forceinline__ uint32_t next_candidate(uint32_t base, double lam, uint32_t hi, uint32_t lo)
{
    if (!(lam > 0.0)) return NEVER;
    double g = ceil(-log(u53(hi, lo)) / lam);
    if (g < 1.0) g = 1.0;
    double t = (double)base + g;
    if (t >= 4294967295.0) return NEVER;
    return (uint32_t)t;
}

// CIC cell and fraction; the clamp keeps z within an ulp of L in the last cell.
__device__ __forceinline__ void cic(double z, double invdz, int N, int &j, double &f)
{
#pragma clang fp contract(off)
    double s = z * invdz;
    double fl = floor(s);
    int jj = (int)fl;
    if (jj < 0) { jj = 0; fl = 0.0; }
    if (jj > N - 1) { jj = N - 1; fl = (double)(N - 1); }
    j = jj;
    f = s - fl;
}

// rne(f 2^32) for f in [0, 1]: the product is exact, the rounded value lies
// in [0, 2^32], and only the end point 2^32 does not fit a 32-bit conversion.
__device__ __forceinline__ unsigned long long fixed_right(double f)
{
#pragma clang fp contract(off)
    const double r = rint(f * TWO32);
    return r >= TWO32 ? (1ull << 32) : (unsigned long long)(unsigned int)r;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide min and max (every thread receives both).
__device__ __forceinline__ void block_minmax(int &mn, int &mx, int *sh)
{
    mn = wave_min(mn);
    mx = wave_max(mx);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { sh[w] = mn; sh[NW + w] = mx; }
    __syncthreads();
    mn = sh[0]; mx = sh[NW];
#pragma unroll
    for (int q = 1; q < NW; ++q) { mn = min(mn, sh[q]); mx = max(mx, sh[NW + q]); }
    __syncthreads();
}


// ---------------------------------------------------------------------------
// Wave-level run reductions.  Cell-sorted particles put long runs of equal
// cells in consecutive lanes; combining each run before touching LDS turns a
// 64-way same-address atomic into one atomic per run.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Segmented inclusive sums of (L, A) over runs of equal key in consecutive
// lanes; 'last' marks the final lane of each run, which then holds the run sums.
__device__ __forceinline__ void run_sums(int key, unsigned long long &L, unsigned long long &A, bool &last)
{
    const int lane = lane_id();
    const int prev = __shfl_up(key, 1, 64);
    const int next = __shfl_down(key, 1, 64);
    int flag = (lane == 0 || prev != key) ? 1 : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long Lo = __shfl_up(L, o, 64), Ao = __shfl_up(A, o, 64);
        const int fo = __shfl_up(flag, o, 64);
        if (lane >= o) {
            if (!flag) { L += Lo; A += Ao; }
            flag |= fo;
        }
    }
    last = (lane == 63) || (next != key);
}

// Start lane and length of the run of equal keys that contains this lane.
__device__ __forceinline__ void run_extent(int key, int &start, int &len)
{
    const int lane = lane_id();
    const int prev = __shfl_up(key, 1, 64);
    const int next = __shfl_down(key, 1, 64);
    int s = (lane == 0 || prev != key) ? lane : 0;
    int e = (lane == 63 || next != key) ? lane : 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(s, o, 64);
        const int u = __shfl_down(e, o, 64);
        if (lane >= o) s = max(s, t);
        if (lane + o < 64) e = min(e, u);
    }
    start = s;
    len = e - s + 1;
}

// ---------------------------------------------------------------------------
// Chunk maps of the particle kernel (tails first, below) and the re-sort.
// ---------------------------------------------------------------------------
// A block-uniform integer (read from LDS or loaded by every lane from one
// address) made a scalar, so that what is derived from it (diode, species,
// buffer pointers, parameters) lives in scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

struct ChunkMap {
    int nseg;
    int total;
};

// Whether a re-sort keeps species s where it is instead of sorting it.  The
// ions move a small fraction of a cell in a re-sort period, so their order
// barely ages: only every ION_SORT_EVERY-th re-sort sorts them, and any
// re-sort does when the tail born since they were last sorted has grown past
// 1/16 of them (a store the host has just written has n_new = 0, all tail) or
// when the free capacity is short (a sort drops the absorbed particles'
// holes).  Decided from the counters as they stand before the re-sort.
constexpr uint32_t ION_SORT_EVERY = 4;
__device__ __forceinline__ bool sort_keeps(const Diode &dd, const DiodeState &st, int s)
{
    if (s != SP_I || st.resorts % ION_SORT_EVERY == 0u) return false;
    const int n = st.n[s], ns = min(max(st.n_new[s], 0), n), tail = n - ns, cap = dd.cap[s];
    return tail <= n / 16 && cap - n >= max(2 * tail, cap / 16);
}

// Segments of the re-sort's chunk map: those it sorts, judged from the
// counters before it (SEGS_SORT_PRE: the count pass, before the scan has
// stored the decision) or as the scan stored it (SEGS_SORT).
enum SegSel { SEGS_SORT_PRE, SEGS_SORT };

__device__ void build_chunk_map(const Diode *__restrict__ D, const DiodeState *__restrict__ S, int nd, int chunk,
                                SegSel sel, int *seg_end, ChunkMap &cm, int *seg_n = nullptr)
{
    int nseg = nd * NSP;
    if (threadIdx.x < 64) {
        int carry = 0;
        for (int b0 = 0; b0 < nseg; b0 += 64) {
            int sidx = b0 + threadIdx.x;
            int c = 0;
            if (sidx < nseg) {
                const DiodeState &st = S[sidx / NSP];
                const int sp = sidx % NSP;
                const int n = st.n[sp];
                const bool kept = sel == SEGS_SORT_PRE ? sort_keeps(D[sidx / NSP], st, sp) : st.keep[sp] != 0;
                c = kept ? 0 : (n + chunk - 1) / chunk;
                if (seg_n) seg_n[sidx] = n;
            }
            // inclusive wave scan
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                int t = __shfl_up(c, o, 64);
                if ((int)threadIdx.x >= o) c += t;
            }
            if (sidx < nseg) seg_end[sidx] = c + carry;
            carry += __shfl(c, 63, 64);
        }
    }
    __syncthreads();
    cm.nseg = nseg;
    cm.total = uni(seg_end[nseg - 1]);
}

__device__ __forceinline__ int find_seg(const int *seg_end, int nseg, int c)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (seg_end[mid] > c) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Chunk order of the particle kernel: the tails of all segments first, then
// their bodies.  A segment's body is its whole chunks below the count the
// last re-sort left (n_new), ordered by bin; its tail is the rest, the
// particles born since (plus the chunk that straddles n_new).  Newborns of
// ionisation lie anywhere in the gap, so a tail run gathers and deposits
// mostly outside its window and costs a block several times a body run: at
// the head of the order such blocks start first and end inside the kernel,
// not after it.  tail_end and body_end are inclusive prefix sums of the
// segments' tail and body chunk counts.
struct TailFirstMap {
    int nseg;
    int ntail;   // tail chunks of all segments
    int total;
};

__device__ void build_tail_first_map(const DiodeState *__restrict__ S, int nd, int chunk, int *tail_end,
                                     int *body_end, int *seg_n, TailFirstMap &cm)
{
    const int nseg = nd * NSP;
    if (threadIdx.x < 64) {
        int carry_t = 0, carry_b = 0;
        for (int b0 = 0; b0 < nseg; b0 += 64) {
            const int sidx = b0 + (int)threadIdx.x;
            int ct = 0, cb = 0;
            if (sidx < nseg) {
                const DiodeState &st = S[sidx / NSP];
                const int n = st.n[sidx % NSP];
                const int ns = min(max(st.n_new[sidx % NSP], 0), n);
                cb = ns / chunk;
                ct = (n + chunk - 1) / chunk - cb;
                seg_n[sidx] = n;
            }
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(ct, o, 64), u = __shfl_up(cb, o, 64);
                if ((int)threadIdx.x >= o) { ct += t; cb += u; }
            }
            if (sidx < nseg) {
                tail_end[sidx] = ct + carry_t;
                body_end[sidx] = cb + carry_b;
            }
            carry_t += __shfl(ct, 63, 64);
            carry_b += __shfl(cb, 63, 64);
        }
    }
    __syncthreads();
    cm.nseg = nseg;
    cm.ntail = uni(tail_end[nseg - 1]);
    cm.total = cm.ntail + uni(body_end[nseg - 1]);
}

// ---------------------------------------------------------------------------
// MCC for one candidate (FP32 kinematics).  Channels are tested in the fixed
// order (e: elastic, excitation, ionisation; ion: charge exchange, elastic);
// a uniform times nu_max picks the first channel whose cumulative frequency
// exceeds it, otherwise the collision is null.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rare_tally_zero(RareTally *t)
{
    // called by thread 0 only, before a barrier
    *t = RareTally{};
}

// vzn: v_z after the push; the position is read back only for an ionization.
__device__ __forceinline__ void mcc_one(const Diode &dd, int s, const GBuf &b, int i, uint32_t step, float vzn,
                                        RareTally *cc)
{
    const int ion = (s == SP_I);
    const ColdRec cr = get_cold(&b.cold[i]);
    float vx = cr.vx, vy = cr.vy, vz = vzn;
    const uint32_t id = cr.id;
    // The three counter blocks are generated one at a time, each consumed
    // before the next (scheduling barriers keep their rounds from being
    // interleaved, which would hold all of them live at once).
    const uint4 C0 = philox(step, EV_COLL, 0u, 0u, id, dd.kseed);
    const float sn = dd.sig_n[ion];
    float a1, a2, a3, a4;
    bm24(C0.x, C0.y, a1, a2);
    bm24(C0.z, C0.w, a3, a4);
    const float vnx = sn * a1, vny = sn * a2, vnz = sn * a3;
    __builtin_amdgcn_sched_barrier(0);
    const uint4 C1 = philox(step, EV_COLL, 1u, 0u, id, dd.kseed);
    const float gx = vx - vnx, gy = vy - vny, gz = vz - vnz;
    const float g2 = gx * gx + gy * gy + gz * gz;
    const float gm = sqrtf(g2);
    const float eps = dd.half_mu_over_e[ion] * g2;          // eV
    const float r = u24f(C1.x) * dd.numax_f[ion];
    const uint32_t ch = dd.channels;
    float cum = 0.0f;
    int taken = -1;
    if (ion) {
        if (ch & (1u << CH_CX)) cum += dd.ng * dd.sig_cx * gm;
        if (taken < 0 && r < cum) taken = CH_CX;
        if (ch & (1u << CH_IEL)) cum += dd.ng * dd.sig_iel * gm;
        if (taken < 0 && r < cum) taken = CH_IEL;
    } else {
        if (ch & (1u << CH_EEL)) cum += dd.ng * dd.sig_el * gm;
        if (taken < 0 && r < cum) taken = CH_EEL;
        if ((ch & (1u << CH_EXC)) && eps > (float)E_EXC) {
            float x = eps * (float)(1.0 / E_EXC);
            cum += dd.ng * (dd.sig_x0 * logf(x) / x) * gm;
        }
        if (taken < 0 && r < cum) taken = CH_EXC;
        if ((ch & (1u << CH_IZ)) && eps > (float)E_ION) {
            cum += dd.ng * (dd.lotz_a2 * logf(eps * (float)(1.0 / E_ION)) / eps) * gm;
        }
        if (taken < 0 && r < cum) taken = CH_IZ;
    }
    if (cum > dd.numax_f[ion]) atomicOr(&dd.st->err, ERR_NULLCOLL);
    __builtin_amdgcn_sched_barrier(0);
    const uint4 C2 = philox(step, EV_COLL, 2u, 0u, id, dd.kseed);
    const uint32_t tcn = next_candidate(step, dd.lam[ion], C2.z, C2.w);
    atomicAdd(&cc->cand[ion], 1u);
    if (taken >= 0) {
        atomicAdd(&cc->coll[taken], 1u);
        const float fm = dd.mfrac_m[ion], fM = dd.mfrac_M[ion];
        const float cx = fm * vx + fM * vnx, cy = fm * vy + fM * vny, cz = fm * vz + fM * vnz;
        if (taken == CH_CX) {
            vx = vnx; vy = vny; vz = vnz;
        } else {
            float ct = 1.0f - 2.0f * u24f(C1.y);
            float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
            float sp, cp;
            sincospif(2.0f * u24f(C1.z), &sp, &cp);
            float gp = gm;
            if (taken == CH_EXC) {
                gp = sqrtf(fmaxf(0.0f, g2 - dd.two_e_over_mu[0] * (float)E_EXC));
            } else if (taken == CH_IZ) {
                float avail = fmaxf(0.0f, eps - (float)E_ION);
                float e1 = u24f(C1.w) * avail;
                float e2 = avail - e1;
                gp = sqrtf(dd.two_e_over_mu[0] * e1);
                float gs = sqrtf(dd.two_e_over_mu[0] * e2);
                float ct2 = 1.0f - 2.0f * u24f(C2.x);
                float st2 = sqrtf(fmaxf(0.0f, 1.0f - ct2 * ct2));
                float sp2, cp2;
                sincospif(2.0f * u24f(C2.y), &sp2, &cp2);
                int q = atomicAdd(&dd.st->iz_count, 1);
                if (q < IZQ_CAP) {
                    IzEvent ev;
                    ev.z = b.z[i];
                    ev.parent = id;
                    ev.ve[0] = cx + fM * gs * st2 * cp2;
                    ev.ve[1] = cy + fM * gs * st2 * sp2;
                    ev.ve[2] = cz + fM * gs * ct2;
                    ev.vi[0] = vnx; ev.vi[1] = vny; ev.vi[2] = vnz;
                    ev.pad = 0;
                    dd.izq[q] = ev;
                } else {
                    atomicOr(&dd.st->err, ERR_IZQ);
                }
            }
            vx = cx + fM * gp * st * cp;
            vy = cy + fM * gp * st * sp;
            vz = cz + fM * gp * ct;
        }
        put_cold(&b.cold[i], vx, vy, id);
        b.vz[i] = vz;
    }
    // a null collision leaves v_z as the push stored it: only the countdown
    // changes (each store here is a partial line written back on its own)
    b.tc[i] = tcn;
}

// ---------------------------------------------------------------------------
// Particle kernel.  mode 0: full step; mode 1: deposit only (load / refield).
//
// Each block owns a contiguous range of chunks; each thread owns PPT
// consecutive slots of a chunk; the re-sort orders them by 32-cell bins.
// Runs of chunks of one (diode, species) share one LDS window: the field tile
// of the gather and the fixed-point histogram of the deposit cover the bins
// of the run's first and last particle plus a drift margin; particles outside
// it use global memory.  The LDS histogram holds one packed word per cell
// (count and sum of a), one LDS atomic per particle, unpacked into node
// values when the run's window is flushed.  A thread sums its consecutive
// same-cell particles in registers and touches LDS only when the cell
// changes; a wave whose lanes end in one cell combines them first.
// Inside a run the chunk loop has no barrier and the next chunk's particle
// data is loaded while the current one is processed.  Rare work (candidates,
// absorbed particles) is queued in LDS and done in batches.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Rare work item: slot index with the kind in the top two bits
// (0 candidate, 1 absorbed at the cathode, 2 absorbed at the anode).  The
// wave's queue keeps the new v_z beside it; items moved to the global list
// re-read v_z from the buffer, stored by the main loop.
constexpr uint32_t RARE_SHIFT = 30;
constexpr uint32_t RARE_MASK = (1u << RARE_SHIFT) - 1u;

template <int PPT>
struct ChunkRegs {
    double z[PPT];
    float vz[PPT];
    uint32_t tc[PPT];
};

// Slots [t0, t0 + PPT) of one thread; capacities are multiples of the largest
// chunk, so the whole range is always inside the buffer.  z and v_z are read
// and written with the non-temporal hint: each line is touched once per step,
// and keeping them from displacing the lines that are reused (field tiles,
// histograms, the collision candidates' records) is worth a fifth of the
// kernel's time.  The countdown is read normally: its lines stay in L2 for
// the candidates' new countdowns, written after the run, to merge into.
template <int PPT>
__device__ __forceinline__ void load_chunk(ChunkRegs<PPT> &C, const GBuf &b, int t0, int mode)
{
#pragma unroll
    for (int k = 0; k < PPT; ++k) C.z[k] = __builtin_nontemporal_load(&b.z[t0 + k]);
    if (mode == 0) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            C.vz[k] = __builtin_nontemporal_load(&b.vz[t0 + k]);
            C.tc[k] = b.tc[t0 + k];
        }
    }
}

// vzn: v_z at the crossing (v^{n+1/2})
__device__ __forceinline__ void rare_absorbed(const Diode &dd, int s, const GBuf &b, int i, int wall, float vzn,
                                              RareTally *rt)
{
    const ColdRec cr = get_cold(&b.cold[i]);
    const double vx = cr.vx, vy = cr.vy, vz = vzn;
    const double ke = 0.5 * dd.mass[s] * (vx * vx + vy * vy + vz * vz);
    atomicAdd(&rt->abs_count[s][wall], 1u);
    atomicAdd(&rt->abs_energy[s][wall], ke);
    if (s == SP_I) atomicAdd(&rt->ion_lost, 1);
}


// The step's rare items of one diode (all species): collisions of candidates,
// tallies of absorbed particles, into the block's LDS tally.  Items
// [first, n) with stride `stride` of each list.
__device__ __forceinline__ void process_rare(const Diode &dd, const int *rare_n, const int *flip, int parity,
                                             uint32_t step, int first, int stride, RareTally *rt)
{
#pragma unroll 1
    for (int s = 0; s < NSP; ++s) {
        const int n = rare_n[s];
        const GBuf b = gbuf(dd.buf[parity ^ flip[s]][s]);
        for (int k = first; k < n; k += stride) {
            const uint32_t item = dd.rare[s][k];
            const int i = (int)(item & RARE_MASK);
            const uint32_t kind = item >> RARE_SHIFT;
            if (kind == 0u) mcc_one(dd, s, b, i, step, b.vz[i], rt);
            else rare_absorbed(dd, s, b, i, (int)kind - 1, b.vz[i], rt);
        }
    }
}

// Add a block-run tally to this block's accumulator copy (device atomics).
__device__ __forceinline__ void flush_tally(const Diode &dd, const RareTally &t)
{
    RareTally &a = dd.tacc[blockIdx.x % TALLY_COPIES].t;
    for (int ion = 0; ion < 2; ++ion)
        if (t.cand[ion]) atomicAdd(&a.cand[ion], t.cand[ion]);
#pragma unroll
    for (int k = 0; k < NCH; ++k)
        if (t.coll[k]) atomicAdd(&a.coll[k], t.coll[k]);
#pragma unroll
    for (int sp = 0; sp < NSP; ++sp)
        for (int w = 0; w < 2; ++w)
            if (t.abs_count[sp][w]) {
                atomicAdd(&a.abs_count[sp][w], t.abs_count[sp][w]);
                atomicAdd(&a.abs_energy[sp][w], t.abs_energy[sp][w]);
            }
    if (t.ion_lost) atomicAdd(&a.ion_lost, t.ion_lost);
}

// Fold the accumulator copies (one per lane of the first wave, read by
// read_tally_copy) into rt (LDS) with a fixed shuffle tree per field.
__device__ __forceinline__ void fold_tally_copies(RareTally v, RareTally *rt)
{
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int k = 0; k < 2; ++k) v.cand[k] += __shfl_xor(v.cand[k], o, 64);
#pragma unroll
        for (int k = 0; k < NCH; ++k) v.coll[k] += __shfl_xor(v.coll[k], o, 64);
#pragma unroll
        for (int sp = 0; sp < NSP; ++sp)
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                v.abs_count[sp][w] += __shfl_xor(v.abs_count[sp][w], o, 64);
                v.abs_energy[sp][w] += __shfl_xor(v.abs_energy[sp][w], o, 64);
            }
        v.ion_lost += __shfl_xor(v.ion_lost, o, 64);
    }
    if (lane == 0) {
        for (int k = 0; k < 2; ++k) rt->cand[k] += v.cand[k];
        for (int k = 0; k < NCH; ++k) rt->coll[k] += v.coll[k];
        for (int sp = 0; sp < NSP; ++sp)
            for (int w = 0; w < 2; ++w) {
                rt->abs_count[sp][w] += v.abs_count[sp][w];
                rt->abs_energy[sp][w] += v.abs_energy[sp][w];
            }
        rt->ion_lost += v.ion_lost;
    }
}

// Add a step's tally to the diode's cumulative tallies (one thread; atomics
// without return, so nothing waits for the old values).
__device__ __forceinline__ void apply_tally(const Diode &dd, const RareTally &t)
{
    DiodeTally *T = dd.tally;
    for (int ion = 0; ion < 2; ++ion)
        if (t.cand[ion]) atomicAdd(&T->cand[ion], (unsigned long long)t.cand[ion]);
#pragma unroll
    for (int k = 0; k < NCH; ++k)
        if (t.coll[k]) atomicAdd(&T->coll[k], (unsigned long long)t.coll[k]);
#pragma unroll
    for (int sp = 0; sp < NSP; ++sp)
        for (int w = 0; w < 2; ++w)
            if (t.abs_count[sp][w]) {
                atomicAdd(&T->abs_count[sp][w], (unsigned long long)t.abs_count[sp][w]);
                atomicAdd(&T->abs_energy[sp][w], t.abs_energy[sp][w]);
            }
}

// The diode's counters, one lane of the calling wave per 32-bit field, read
// at agent scope (other kernels' atomics land in L2).
__device__ __forceinline__ void load_state(const DiodeState *st, DiodeState *out)
{
    constexpr int W = (int)(sizeof(DiodeState) / 4);
    static_assert(W <= 64, "one lane per field");
    const int lane = threadIdx.x & 63;
    if (lane < W)
        reinterpret_cast<uint32_t *>(out)[lane] = __hip_atomic_load(
            glb(reinterpret_cast<const uint32_t *>(st)) + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Packed deposit word of cell j: (particle count << PK_SHIFT) + sum of a.
// The cell's particles give node j  count * 2^32 - sum a  and node j+1  sum a,
// so one word per cell carries both.  A run holds at most RUN_PARTICLES
// particles, so the sum of a (each <= 2^32) stays below 2^PK_SHIFT and the
// count below 2^(64 - PK_SHIFT).
constexpr int PK_SHIFT = 48;
constexpr unsigned long long PK_MASK = (1ull << PK_SHIFT) - 1ull;
constexpr int RUN_PARTICLES = 65535;

// Add a packed cell word to the LDS window when the cell is inside it, else
// its two node contributions to global memory.
__device__ __forceinline__ void flush_run(int j, unsigned long long P, int w0, int wn,
                                          unsigned long long *hist, GLB unsigned long long *H)
{
    const int jl = j - w0;
    if (jl >= 0 && jl + 1 < wn) {
        atomicAdd(&hist[jl], P);
    } else {
        const unsigned long long A = P & PK_MASK;
        const unsigned long long L = ((P >> PK_SHIFT) << 32) - A;
        if (L) gadd(&H[j], L);
        if (A) gadd(&H[j + 1], A);
    }
}

#ifndef PIC_PARTICLE_MIN_WAVES
#define PIC_PARTICLE_MIN_WAVES 1
#endif
template <int PPT>
__global__ __launch_bounds__(NT, PIC_PARTICLE_MIN_WAVES) void k_particles(const Diode *__restrict__ D, const DiodeState *__restrict__ S,
                                                  int nd, int mode, int parity)
{
    constexpr int CHUNK = NT * PPT;
    constexpr int RUN_CHUNKS = RUN_PARTICLES / CHUNK < 1 ? 1 : RUN_PARTICLES / CHUNK;   // chunks per run at most
    extern __shared__ int seg_dyn[];    // tail_end, body_end, seg_n: NSP * nd each
    int *tail_end = seg_dyn, *body_end = seg_dyn + NSP * nd, *seg_n = seg_dyn + 2 * NSP * nd;
    __shared__ double etile[WMAX + 2];
    __shared__ unsigned long long hist[WMAX + 2];
    constexpr int QW = 64 * PPT + QW_SLACK;
    __shared__ uint32_t rq_i[NW][QW];   // slot | kind << 30
    __shared__ float rq_v[NW][QW];      // v_z after the push
    __shared__ int q_n[NW];
    __shared__ RareTally rt;

    if (threadIdx.x == 0) rare_tally_zero(&rt);
    TailFirstMap cm;
    build_tail_first_map(S, nd, CHUNK, tail_end, body_end, seg_n, cm);
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63;
    const int per_block = (cm.total + gridDim.x - 1) / gridDim.x;
    const int v_begin = blockIdx.x * per_block;
    const int v_end = min(cm.total, v_begin + per_block);

    for (int v = v_begin; v < v_end;) {
        // the run: chunks [p0, p0 + nrun) of one segment's tail or body
        const bool tail = v < cm.ntail;
        int seg, p0, avail;
        if (tail) {
            seg = uni(find_seg(tail_end, cm.nseg, v));
            const int tb = seg ? tail_end[seg - 1] : 0;
            p0 = uni(body_end[seg] - (seg ? body_end[seg - 1] : 0) + v - tb);
            avail = uni(tail_end[seg] - v);
        } else {
            const int u = v - cm.ntail;
            seg = uni(find_seg(body_end, cm.nseg, u));
            p0 = uni(u - (seg ? body_end[seg - 1] : 0));
            avail = uni(body_end[seg] - u);
        }
        const int nrun = uni(min(min(v_end - v, avail), RUN_CHUNKS));
        const int d = seg / NSP, s = seg - d * NSP;
        const Diode &dd = D[d];
        const GBuf b = gbuf(dd.buf[parity ^ uni(S[d].flip[s])][s]);
        const int N = dd.N;
        const double invdz = dd.invdz;
        const int n = uni(seg_n[seg]);
        const int slot0 = p0 * CHUNK;

        const uint32_t step = (uint32_t)uni((int)S[d].step);
        // the run's first chunk is loaded while the window and field tile are set up
        ChunkRegs<PPT> A, Bn;
        load_chunk<PPT>(A, b, slot0 + tid * PPT, mode);
        // window of the run from its first and last particle (scalar loads,
        // in flight with the chunk); a hole (an absorbed particle, z < 0) at
        // one end gives way to the other end
        const int p_end = p0 + nrun;
        int w0, wn;
        {
            double za = b.z[slot0], zb = b.z[min(n, p_end * CHUNK) - 1];
            if (za < 0.0) za = zb;
            if (zb < 0.0) zb = za;
            int ja, jb;
            double f;
            cic(za, invdz, N, ja, f);
            cic(zb, invdz, N, jb, f);
            // the re-sort orders by bins: the run spans whole bins between its ends
            const int ba = min(ja, jb) >> BIN_SHIFT, bb = max(ja, jb) >> BIN_SHIFT;
            w0 = uni(max(0, (ba << BIN_SHIFT) - DRIFT));
            wn = uni(min(min(N, ((bb + 1) << BIN_SHIFT) + DRIFT) - w0 + 1, WMAX + 1));
        }
        // the large-grid field step leaves E short by one uniform shift per diode
        const double eshift = S[d].e_shift;
        for (int t = tid; t < wn; t += NT) {
            if (mode == 0) etile[t] = glb(dd.E)[w0 + t] + eshift;
            hist[t] = 0ull;
        }
        lds_barrier();

        const double qmdt = dd.qmdt[s], dt = dd.dt, L = dd.L;
        GLB unsigned long long *H = glb(dd.H[s]);
        // The chunks of the run have no barrier: each wave streams its share of
        // every chunk, holding the next chunk's particle registers in flight
        // while it works on the current one.  Rare items (collision candidates,
        // absorbed particles) go to the wave's LDS queue and are done by the
        // whole block after the run.  A wave whose queue could overflow moves
        // its items to the species' list in global memory instead, which the
        // sources kernels work through.
        GLB uint32_t *rare = glb(dd.rare[s]);
        int qn = 0;     // the wave's queue length (wave-uniform)
        // The z, v_z stores of a chunk are issued one iteration later, after the
        // next prefetch: loads and stores share one completion counter whose
        // order between the two kinds is not kept, so the wait for the
        // prefetched registers also waits for every store issued before it.
        double zs[PPT];
        float vs[PPT];
        int ts = -1;
        for (int pc = p0; pc < p_end; ++pc) {
            if (mode == 0 && qn > QW - 64 * PPT) {
                int base = 0;
                if (lane == 0)
                    base = __hip_atomic_fetch_add(glb(&dd.st->rare_n[s]), qn, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
                base = __shfl(base, 0, 64);
                for (int q = lane; q < qn; q += 64) rare[base + q] = rq_i[w][q];
                qn = 0;
            }
            const int t0 = pc * CHUNK + tid * PPT;
            if (pc + 1 < p_end) load_chunk<PPT>(Bn, b, t0 + CHUNK, mode);
            if (mode == 0 && ts >= 0) {
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    __builtin_nontemporal_store(zs[k], &b.z[ts + k]);
                    __builtin_nontemporal_store(vs[k], &b.vz[ts + k]);
                }
            }
            int jcur = -1;
            unsigned long long accP = 0ull;
            double zw[PPT];
            float vw[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int i = t0 + k;
                bool alive = i < n && A.z[k] >= 0.0;
                uint32_t item = NEVER;
                double z = A.z[k];
                zw[k] = A.z[k];
                vw[k] = A.vz[k];
                if (alive && mode == 0) {
                    int jo;
                    double fo;
                    cic(z, invdz, N, jo, fo);
                    const int jl = jo - w0;
                    const bool inw = jl >= 0 && jl + 1 < wn;
                    double Ep;
                    if (__builtin_expect(__ballot(!inw) != 0ull, 0)) {
                        // a lane outside the window: this wave reads E from global
                        // memory and waits for it here, so the common path below
                        // carries no wait on a global load (which would also wait
                        // for the next chunk's prefetch)
                        double e0, e1;
                        if (inw) { e0 = etile[jl]; e1 = etile[jl + 1]; }
                        else { e0 = glb(dd.E)[jo] + eshift; e1 = glb(dd.E)[jo + 1] + eshift; }
                        {
#pragma clang fp contract(off)
                            Ep = (1.0 - fo) * e0 + fo * e1;
                        }
                        asm volatile("" : "+v"(Ep));
                    } else {
#pragma clang fp contract(off)
                        Ep = (1.0 - fo) * etile[jl] + fo * etile[jl + 1];
                    }
                    const float vzn = (float)((double)A.vz[k] + qmdt * Ep);
                    const double zn = z + (double)vzn * dt;
                    vw[k] = vzn;
                    if (zn <= 0.0 || zn >= L) {
                        // absorbing electrodes: tallied with the rare work
                        zw[k] = -1.0;
                        alive = false;
                        item = (uint32_t)i | ((zn <= 0.0 ? 1u : 2u) << RARE_SHIFT);
                    } else {
                        if (!(zn == zn))
                            __hip_atomic_fetch_or(glb(&dd.st->err), (unsigned)ERR_NAN, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
                        z = zn;
                        zw[k] = zn;
                        if (A.tc[k] == step) item = (uint32_t)i;
                    }
                }
                if (mode == 0) {
                    // append to the wave's queue: slot from the ballot, no LDS atomics
                    const unsigned long long m = __ballot(item != NEVER);
                    if (m) {
                        const int pos = qn + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        if (item != NEVER) {
                            rq_i[w][pos] = item;
                            rq_v[w][pos] = vw[k];
                        }
                        qn = uni(qn + __popcll(m));
                    }
                }
                if (alive) {
                    int j;
                    double f;
                    cic(z, invdz, N, j, f);
                    const unsigned long long p = (1ull << PK_SHIFT) + fixed_right(f);
                    if (j != jcur) {
                        if (jcur >= 0) flush_run(jcur, accP, w0, wn, hist, H);
                        jcur = j;
                        accP = p;
                    } else {
                        accP += p;
                    }
                }
            }
            if (mode == 0) {
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    zs[k] = zw[k];
                    vs[k] = vw[k];
                }
                ts = t0;
            }
            // last run of every lane: combine across the wave when all lanes agree
            const int j0w = __shfl(jcur, 0, 64);
            if (__all(jcur == j0w)) {
                const unsigned long long sP = wave_sum_u64(accP);
                if (lane == 0 && j0w >= 0) flush_run(j0w, sP, w0, wn, hist, H);
            } else if (jcur >= 0) {
                flush_run(jcur, accP, w0, wn, hist, H);
            }
            A = Bn;
        }
        if (mode == 0 && ts >= 0) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                __builtin_nontemporal_store(zs[k], &b.z[ts + k]);
                __builtin_nontemporal_store(vs[k], &b.vz[ts + k]);
            }
        }
        if (lane == 0) q_n[w] = qn;
        // the main loop's z, v_z stores precede the rare work's reads (workgroup scope)
        __syncthreads();
        // node w0 + t: cell t's  count * 2^32 - sum a  plus cell t-1's  sum a
        for (int t = tid; t < wn; t += NT) {
            const unsigned long long P = hist[t];
            const unsigned long long Pm = t > 0 ? hist[t - 1] : 0ull;
            const unsigned long long v = ((P >> PK_SHIFT) << 32) - (P & PK_MASK) + (Pm & PK_MASK);
            if (v) gadd(&H[w0 + t], v);
        }
        if (mode == 0) {
            // the run's rare items with the whole block, soon after the run
            // (the countdown lines are still in L2): collisions of candidates, tallies of absorbed
            int tot = 0;
#pragma unroll
            for (int q = 0; q < NW; ++q) tot += q_n[q];
            for (int q = tid; q < tot; q += NT) {
                int wq = 0, k = q;
                while (k >= q_n[wq]) { k -= q_n[wq]; ++wq; }
                const uint32_t item = rq_i[wq][k];
                const int i = (int)(item & RARE_MASK);
                const uint32_t kind = item >> RARE_SHIFT;
                if (kind == 0u) mcc_one(dd, s, b, i, step, rq_v[wq][k], &rt);
                else rare_absorbed(dd, s, b, i, (int)kind - 1, rq_v[wq][k], &rt);
            }
            lds_barrier();
            if (tid == 0) {
                flush_tally(dd, rt);
                rare_tally_zero(&rt);
            }
        }
        lds_barrier();
        v += nrun;
    }
}

// ---------------------------------------------------------------------------
// Initial load ("Model": uniform positions, Maxwellian velocities, no drift).
// grid: (ceil(n_load_max / 256), nd, 2); z selects electrons (0) or ions (1).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_load(const Diode *__restrict__ D, const long long *n_load)
{
    const int d = blockIdx.y;
    const int s = blockIdx.z == 0 ? SP_P : SP_I;
    const long long nl = n_load[d];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= nl) return;
    const Diode &dd = D[d];
    const uint32_t id = (uint32_t)(s == SP_P ? i : nl + i);
    uint4 b0 = philox(LOAD_STEP, EV_LOAD, 0u, 0u, id, dd.kseed);
    uint4 b1 = philox(LOAD_STEP, EV_LOAD, 1u, 0u, id, dd.kseed);
    double n1, n2, n3, n4;
    bm32(b0.x, b0.y, n1, n2);
    bm32(b0.z, b0.w, n3, n4);
    const double sig = s == SP_P ? dd.sig_e0 : dd.sig_i0;
    const GBuf b = gbuf(dd.buf[0][s]);
    b.z[i] = dd.L * u53(b1.x, b1.y);
    put_cold(&b.cold[i], (float)(sig * n1), (float)(sig * n2), id);
    b.vz[i] = (float)(sig * n3);
    uint32_t tc = next_candidate(0u, dd.lam[s == SP_I], b1.z, b1.w);
    if (tc != NEVER) tc -= 1u;
    b.tc[i] = tc;
}

// ---------------------------------------------------------------------------
// Warm start from cell-centre density profiles.  dens[d][q][c] (q = 0
// electrons, 1 ions; rows of max_cells doubles).  Cell c of species q holds
// floor(x) particles plus one with probability frac(x), x = n dz / w0, the
// Bernoulli draw keyed by the cell.  One block per diode writes the exclusive
// cell offsets (N + 1 entries) into the re-sort's count array, the live
// counts and the next id; errors are sticky bits that skip the fill.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_profile_count(const Diode *__restrict__ D, const double *__restrict__ dens,
                                                        int rows, int max_cells)
{
    const Diode &dd = D[blockIdx.x];
    const int N = dd.N, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    __shared__ long long wsum[16];
    __shared__ long long base_s;
    __shared__ int bad;
    if (tid == 0) bad = 0;
    long long tot[2];
    for (int q = 0; q < 2; ++q) {
        const int s = q == 0 ? SP_P : SP_I;
        const double *n = dens + ((size_t)blockIdx.x * rows + q) * max_cells;
        int *off = dd.cell_cnt[s];
        if (tid == 0) base_s = 0;
        __syncthreads();
        for (int c0 = 0; c0 < N; c0 += 1024) {
            const int c = c0 + tid;
            long long cnt = 0;
            if (c < N) {
                const double x = n[c] * dd.dz / dd.w0;
                if (!(x >= 0.0) || x > 1073741824.0) {
                    bad = 1;
                } else {
                    const double fl = floor(x);
                    const uint4 r = philox(LOAD_STEP, EV_PROFILE, (uint32_t)q, 0u, (uint32_t)c, dd.kseed);
                    cnt = (long long)fl + (u53(r.x, r.y) < x - fl ? 1 : 0);
                }
            }
            long long inc = cnt;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const long long t = __shfl_up(inc, o, 64);
                if (lane >= o) inc += t;
            }
            if (lane == 63) wsum[w] = inc;
            __syncthreads();
            long long wb = base_s;
            for (int k = 0; k < w; ++k) wb += wsum[k];
            const long long excl = wb + inc - cnt;
            if (c < N) off[c] = (int)min(excl, 0x7FFFFFFFll);
            __syncthreads();
            if (tid == 1023) base_s = excl + cnt;
            __syncthreads();
        }
        tot[q] = base_s;
        if (tid == 0) off[N] = (int)min(base_s, 0x7FFFFFFFll);
        __syncthreads();
    }
    if (tid == 0) {
        DiodeState *st = dd.st;
        uint32_t err = 0;
        if (bad) err |= ERR_NAN;
        if (tot[0] > dd.cap[SP_P] || tot[1] > dd.cap[SP_I] || tot[0] + tot[1] > 0xFFFF0000ll) err |= ERR_CAPACITY;
        st->n[SP_E] = 0;
        if (err) {
            st->err |= err;
            st->n[SP_P] = st->n[SP_I] = 0;
            st->next_id = 0;
        } else {
            st->n[SP_P] = (int32_t)tot[0];
            st->n[SP_I] = (int32_t)tot[1];
            st->next_id = (uint32_t)(tot[0] + tot[1]);
        }
    }
}

// Quantile levels of the state load's velocity summaries.
__constant__ double QLEV[9] = {0.0, 0.02, 0.1, 0.25, 0.5, 0.75, 0.9, 0.98, 1.0};

// Sampling from nine quantiles: sorted first (so an unordered prediction is
// read as its monotone rearrangement), then inverted piecewise-linearly.
__device__ __forceinline__ void sort_q9(double q[9])
{
#pragma unroll
    for (int i = 1; i < 9; ++i)
#pragma unroll
        for (int j = 8; j >= i; --j) {
            const double lo = fmin(q[j - 1], q[j]), hi = fmax(q[j - 1], q[j]);
            q[j - 1] = lo;
            q[j] = hi;
        }
}
__device__ __forceinline__ double from_q9(const double q[9], double u)
{
    int k = 0;
#pragma unroll
    for (int m = 1; m < 8; ++m) k += (u >= QLEV[m]) ? 1 : 0;
    const double t = (u - QLEV[k]) / (QLEV[k + 1] - QLEV[k]);
    double lo = q[0], hi = q[1];
#pragma unroll
    for (int m = 1; m < 8; ++m)
        if (k == m) { lo = q[m]; hi = q[m + 1]; }
    return lo + t * (hi - lo);
}

// One wave per (cell, species): the cell's particles, keyed by id as in the
// uniform load, positions uniform in the cell.  state == null: velocities
// Maxwellian at the load temperature, drawn as in the uniform load.  Else
// state [diode][STATE_ROWS][max_cells]: v_z and |v_perp| from the cell's
// quantiles (rows 3 + 18 q and 12 + 18 q, q = 0 electrons, 1 ions), a uniform
// azimuth, and the kinetic energy limited to load_cap_ev (the null-collision
// bound's energy cap).
__global__ __launch_bounds__(256) void k_profile_fill(const Diode *__restrict__ D, const double *__restrict__ state,
                                                      int max_cells)
{
    const Diode &dd = D[blockIdx.y];
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int q = blockIdx.z;
    const int s = q == 0 ? SP_P : SP_I;
    if (c >= dd.N || dd.st->err) return;
    const int *off = dd.cell_cnt[s];
    const int a = off[c], e = off[c + 1];
    const uint32_t id0 = s == SP_P ? 0u : (uint32_t)dd.cell_cnt[SP_P][dd.N];
    const double sig = s == SP_P ? dd.sig_e0 : dd.sig_i0;
    const double lam = dd.lam[s == SP_I];
    const GBuf b = gbuf(dd.buf[0][s]);
    double qz[9], qp[9], emax = 0.0;
    if (state) {
        const double *row = state + (size_t)blockIdx.y * STATE_ROWS * max_cells + c;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            qz[k] = row[(size_t)(3 + 18 * q + k) * max_cells];
            qp[k] = row[(size_t)(12 + 18 * q + k) * max_cells];
        }
        bool fin = isfinite(row[(size_t)2 * max_cells]);
#pragma unroll
        for (int k = 0; k < 9; ++k) fin = fin && isfinite(qz[k]) && isfinite(qp[k]);
        if (!fin) {
            if (lane == 0) atomicOr(&dd.st->err, ERR_NAN);
            return;
        }
        sort_q9(qz);
        sort_q9(qp);
        emax = Q_E * dd.load_cap_ev[q];
    }
    for (int i = a + lane; i < e; i += 64) {
        const uint32_t id = id0 + (uint32_t)i;
        const uint4 b0 = philox(LOAD_STEP, EV_LOAD, 0u, 0u, id, dd.kseed);
        const uint4 b1 = philox(LOAD_STEP, EV_LOAD, 1u, 0u, id, dd.kseed);
        double vx, vy, vz;
        if (state) {
            const uint4 b2 = philox(LOAD_STEP, EV_LOAD, 2u, 0u, id, dd.kseed);
            vz = from_q9(qz, u53(b0.x, b0.y));
            const double vp = fmax(0.0, from_q9(qp, u53(b0.z, b0.w)));
            double sa, ca;
            sincospi(2.0 * u53(b2.x, b2.y), &sa, &ca);
            vx = vp * ca;
            vy = vp * sa;
            const double ke = 0.5 * dd.mass[s] * (vx * vx + vy * vy + vz * vz);
            if (ke > emax) {
                const double f = emax > 0.0 ? sqrt(emax / ke) : 0.0;
                vx *= f;
                vy *= f;
                vz *= f;
            }
        } else {
            double n1, n2, n3, n4;
            bm32(b0.x, b0.y, n1, n2);
            bm32(b0.z, b0.w, n3, n4);
            vx = sig * n1;
            vy = sig * n2;
            vz = sig * n3;
        }
        b.z[i] = ((double)c + u53(b1.x, b1.y)) * dd.dz;
        put_cold(&b.cold[i], (float)vx, (float)vy, id);
        b.vz[i] = (float)vz;
        uint32_t tc = next_candidate(0u, lam, b1.z, b1.w);
        if (tc != NEVER) tc -= 1u;
        b.tc[i] = tc;
    }
}

// The re-sort expects its count array zeroed.
__global__ __launch_bounds__(256) void k_profile_clear(const Diode *__restrict__ D)
{
    const Diode &dd = D[blockIdx.x];
    for (int j = threadIdx.x; j <= dd.N; j += 256) {
        dd.cell_cnt[SP_P][j] = 0;
        dd.cell_cnt[SP_I][j] = 0;
    }
}

// ---------------------------------------------------------------------------
// Phase-space histogram ("Phase-space and velocity-distribution
// characteristics"): live particles of one species of one diode counted per
// (z, v_z) bin.  Row iz = min(nz - 1, floor(z sz)), sz = nz / L; with
// x = (v_z - vmin) sv, sv = nv / (vmax - vmin): column 0 for x < 0, 1 + floor(x)
// for 0 <= x < nv, nv + 1 for x >= nv.  Each block counts a contiguous slot
// range (a narrow range of cells once sorted) in LDS and adds its nonzero bins
// to the caller's uint64 counts.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_phase_hist(const Diode *__restrict__ D, const DiodeState *__restrict__ S,
                                                    int d, int s, int parity, int nz, int nv, double sz, double vmin,
                                                    double sv, unsigned long long *__restrict__ out)
{
    extern __shared__ uint32_t ph_hist[];
    const int W = nv + 2, nb = nz * W, tid = threadIdx.x;
    for (int i = tid; i < nb; i += 256) ph_hist[i] = 0u;
    const Diode &dd = D[d];
    const GBuf b = gbuf(dd.buf[parity ^ S[d].flip[s]][s]);
    const int n = S[d].n[s];
    const int per = (n + (int)gridDim.x - 1) / (int)gridDim.x;
    const int i0 = (int)blockIdx.x * per, i1 = min(n, i0 + per);
    __syncthreads();
    for (int i = i0 + tid; i < i1; i += 256) {
        const double z = b.z[i];
        if (!(z >= 0.0)) continue;                     // hole
        const int iz = min(nz - 1, (int)(z * sz));
        const double x = ((double)b.vz[i] - vmin) * sv;
        const int iv = x >= (double)nv ? nv + 1 : (x >= 0.0 ? 1 + (int)x : 0);
        atomicAdd(&ph_hist[iz * W + iv], 1u);
    }
    __syncthreads();
    for (int i = tid; i < nb; i += 256) {
        const uint32_t c = ph_hist[i];
        if (c) atomicAdd(&out[i], (unsigned long long)c);
    }
}

extern "C" hipError_t picx_launch_phase_hist(const Diode *D, const DiodeState *S, int d, int s, int parity, int nz,
                                             int nv, double sz, double vmin, double sv, unsigned long long *out,
                                             int blocks, hipStream_t st)
{
    const size_t lds = (size_t)nz * (nv + 2) * sizeof(uint32_t);
    hipLaunchKernelGGL(k_phase_hist, dim3(blocks), dim3(256), lds, st, D, S, d, s, parity, nz, nv, sz, vmin, sv,
                       out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Re-sort by bins of 32 cells: count -> scan -> scatter -> finalize (compacts
// holes too).  Bins rather than cells: the LDS windows only need each run of
// chunks confined to a narrow range of cells, and with electrons drifting
// tens of cells between re-sorts a chunk then writes a few long destination
// ranges instead of a hundred short ones.
// ---------------------------------------------------------------------------
// Wave-level grouping of equal keys (key < 0: no item).  For each distinct
// key the lowest lane adds the group size to the counter `add` picks (LDS
// window or global) and every member gets that atomic's old value plus its
// rank among the group's lanes.  With few distinct keys per wave (the
// re-sort's bins) this is one atomic per key instead of one per lane.
template <class AddFn>
__device__ __forceinline__ int wave_group_rank(int key, AddFn add)
{
    const int lane = lane_id();
    const bool valid = key >= 0;
    unsigned long long todo = __ballot(valid);
    int rank = 0;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int kl = __shfl(key, leader, 64);
        const unsigned long long m = __ballot(valid && key == kl);
        int base = 0;
        if (lane == leader) base = add(kl, __popcll(m));
        base = __shfl(base, leader, 64);
        if (valid && key == kl)
            rank = base + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        todo &= ~m;
    }
    return rank;
}

// Window of a run of chunks for the re-sort: every bin of the grid when they
// fit the LDS counts, else the bins of the run's first and last particle plus
// the re-sort's drift margin.
__device__ __forceinline__ void sort_window(const Diode &dd, const GBuf &b, int slot0, int last_slot, int &w0,
                                            int &wn)
{
    const int nb = nbins_of(dd.N);
    if (nb <= WMAX + 1) {
        // every bin of the grid fits the LDS counts (N <= 16416): nothing falls outside
        w0 = 0;
        wn = nb;
        return;
    }
    int ja, jb;
    double f;
    cic(b.z[slot0], dd.invdz, dd.N, ja, f);
    cic(b.z[max(last_slot, slot0)], dd.invdz, dd.N, jb, f);
    ja >>= BIN_SHIFT;
    jb >>= BIN_SHIFT;
    w0 = uni(max(0, min(ja, jb) - SORT_DRIFT_B));
    wn = uni(min(min(nbins_of(dd.N) - 1, max(ja, jb) + SORT_DRIFT_B) - w0 + 1, WMAX + 1));
}

// Cell counts of the live particles.  Each thread counts runs of equal cells
// over its PPT consecutive slots and adds them to the block's LDS window.
template <int PPT>
__global__ __launch_bounds__(NT) void k_sort_count(const Diode *__restrict__ D, const DiodeState *__restrict__ S,
                                                   int nd, int parity)
{
    constexpr int CHUNK = NT * PPT;
    __shared__ int seg_end[NSP * MAX_DIODES];
    __shared__ int seg_n[NSP * MAX_DIODES];
    __shared__ int cnt[WMAX + 2];
    ChunkMap cm;
    build_chunk_map(D, S, nd, CHUNK, SEGS_SORT_PRE, seg_end, cm, seg_n);
    const int tid = threadIdx.x;
    const int per_block = (cm.total + gridDim.x - 1) / gridDim.x;
    const int c_begin = blockIdx.x * per_block;
    const int c_end = min(cm.total, c_begin + per_block);
    for (int c = c_begin; c < c_end;) {
        const int seg = find_seg(seg_end, cm.nseg, c);
        const int run_end = min(c_end, seg_end[seg]);
        const int segbase = seg ? seg_end[seg - 1] : 0;
        const int d = seg / NSP, s = seg - d * NSP;
        const Diode &dd = D[d];
        const GBuf b = gbuf(dd.buf[parity ^ S[d].flip[s]][s]);
        const int n = seg_n[seg];
        const int slot0 = (c - segbase) * CHUNK;
        int w0, wn;
        sort_window(dd, b, slot0, min(n, (run_end - segbase) * CHUNK) - 1, w0, wn);
        // the next chunk's positions are in flight while a chunk is counted
        double zn[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) zn[k] = b.z[slot0 + tid * PPT + k];
        for (int t = tid; t < wn; t += NT) cnt[t] = 0;
        lds_barrier();
        GLB int *gc = glb(dd.cell_cnt[s]);
        auto add = [&](int key, int m) {
            const int jl = key - w0;
            if (jl >= 0 && jl < wn) atomicAdd(&cnt[jl], m);
            else gadd(&gc[bin_slot(key)], m);
            return 0;
        };
        for (int cc_ = c; cc_ < run_end; ++cc_) {
            const int t0 = (cc_ - segbase) * CHUNK + tid * PPT;
            double zc[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) zc[k] = zn[k];
            if (cc_ + 1 < run_end) {
#pragma unroll
                for (int k = 0; k < PPT; ++k) zn[k] = b.z[t0 + CHUNK + k];
            }
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                int j = -1;
                if (t0 + k < n && zc[k] >= 0.0) {
                    double f;
                    cic(zc[k], dd.invdz, dd.N, j, f);
                    j >>= BIN_SHIFT;
                }
                wave_group_rank(j, add);
            }
        }
        lds_barrier();
        for (int t = tid; t < wn; t += NT)
            if (cnt[t]) gadd(&gc[bin_slot(w0 + t)], cnt[t]);
        lds_barrier();
        c = run_end;
    }
}

// One workgroup per (diode, species): exclusive scan of the bin counts.
__global__ __launch_bounds__(1024) void k_sort_scan(const Diode *__restrict__ D)
{
    __shared__ int part[1024];
    const int d = blockIdx.x / NSP, s = blockIdx.x % NSP;
    const Diode &dd = D[d];
    // the decision of the count pass, from the same counters, stored for the
    // scatter and the finalize (this block writes n_new[s] below)
    const bool kept = sort_keeps(dd, *dd.st, s);
    if (threadIdx.x == 0) dd.st->keep[s] = kept ? 1 : 0;
    if (kept) return;
    const int N = nbins_of(dd.N);
    int *cc = dd.cell_cnt[s];
    const int per = (N + 1023) / 1024;
    const int j0 = threadIdx.x * per;
    int local = 0;
    for (int j = j0; j < min(N, j0 + per); ++j) local += cc[bin_slot(j)];
    part[threadIdx.x] = local;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int v = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = part[threadIdx.x] - local;
    for (int j = j0; j < min(N, j0 + per); ++j) {
        int v = cc[bin_slot(j)];
        cc[bin_slot(j)] = run;
        run += v;
    }
    if (threadIdx.x == 1023) dd.st->n_new[s] = part[1023];
}

// Scatter into the other buffer in bin order (holes dropped).  A block takes
// its contiguous range of chunks run by run (a run lies in one diode and
// species): it counts the run's particles per bin of the run's window in LDS,
// reserves one contiguous range per bin with one global atomic each, then
// streams the run again and gives every particle the next slot of its bin's
// range from an LDS atomic.  A bin's particles of the run so leave as one
// contiguous range written by one block (its lines fill in L2 before they are
// written back), and the stream needs no barrier.  A particle outside the
// window (a newborn of the unsorted tail, say) takes a slot from its bin's
// global counter directly.
template <int PPT>
__global__ __launch_bounds__(NT) void k_sort_scatter(const Diode *__restrict__ D, const DiodeState *__restrict__ S,
                                                     int nd, int parity)
{
    constexpr int CHUNK = NT * PPT;
    __shared__ int seg_end[NSP * MAX_DIODES];
    __shared__ int seg_n[NSP * MAX_DIODES];
    __shared__ int cur[WMAX + 2];       // the run's count per window bin, then its next free slot
    ChunkMap cm;
    build_chunk_map(D, S, nd, CHUNK, SEGS_SORT, seg_end, cm, seg_n);
    const int tid = threadIdx.x;
    const int per_block = (cm.total + gridDim.x - 1) / gridDim.x;
    const int c_begin = blockIdx.x * per_block;
    const int c_end = min(cm.total, c_begin + per_block);
    for (int c = c_begin; c < c_end;) {
        const int seg = find_seg(seg_end, cm.nseg, c);
        const int run_end = min(c_end, seg_end[seg]);
        const int segbase = seg ? seg_end[seg - 1] : 0;
        const int d = seg / NSP, s = seg - d * NSP;
        const Diode &dd = D[d];
        const int bsel = parity ^ S[d].flip[s];
        const GBuf src = gbuf(dd.buf[bsel][s]);
        const GBuf dst = gbuf(dd.buf[bsel ^ 1][s]);
        const int n = seg_n[seg];
        const int slot0 = (c - segbase) * CHUNK;
        const int slot_end = min(n, (run_end - segbase) * CHUNK);
        int w0, wn;
        sort_window(dd, src, slot0, slot_end - 1, w0, wn);
        for (int t = tid; t < wn; t += NT) cur[t] = 0;
        GLB int *gc = glb(dd.cell_cnt[s]);
        auto bin_of = [&](double z) {
            int j;
            double f;
            cic(z, dd.invdz, dd.N, j, f);
            j >>= BIN_SHIFT;
            return j;
        };
        // the run's first chunk of records is in flight through the count
        double zq[PPT];
        float vq[PPT];
        u32x4 cq[PPT];
        uint32_t tq[PPT];
        auto fetch = [&](int t0) {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                zq[k] = -1.0;
                if (t0 + k < slot_end) {
                    zq[k] = src.z[t0 + k];
                    vq[k] = src.vz[t0 + k];
                    cq[k] = *(const GLB u32x4 *)&src.cold[t0 + k];
                    tq[k] = src.tc[t0 + k];
                }
            }
        };
        fetch(slot0 + tid * PPT);
        lds_barrier();
        // pass 1: the run's counts per window bin (positions one chunk ahead)
        {
            double zn[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int t = slot0 + tid * PPT + k;
                zn[k] = t < slot_end ? src.z[t] : -1.0;
            }
            for (int t0 = slot0 + tid * PPT; t0 < slot_end; t0 += CHUNK) {
                double zc[PPT];
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    zc[k] = zn[k];
                    const int t = t0 + CHUNK + k;
                    zn[k] = t < slot_end ? src.z[t] : -1.0;
                }
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    if (zc[k] < 0.0) continue;
                    const int jl = bin_of(zc[k]) - w0;
                    if (jl >= 0 && jl < wn) atomicAdd(&cur[jl], 1);
                }
            }
        }
        lds_barrier();
        // one contiguous range per bin of the window
        for (int t = tid; t < wn; t += NT) {
            const int v = cur[t];
            if (v) cur[t] = gadd(&gc[bin_slot(w0 + t)], v);
        }
        lds_barrier();
        // pass 2: every particle to the next slot of its bin's range
        for (int t0 = slot0 + tid * PPT; t0 < slot_end; t0 += CHUNK) {
            double z[PPT];
            float vzr[PPT];
            u32x4 cold[PPT];
            uint32_t tcr[PPT];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                z[k] = zq[k];
                vzr[k] = vq[k];
                cold[k] = cq[k];
                tcr[k] = tq[k];
            }
            if (t0 + CHUNK < slot_end) fetch(t0 + CHUNK);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (z[k] < 0.0) continue;
                const int j = bin_of(z[k]), jl = j - w0;
                const int dest = (jl >= 0 && jl < wn) ? atomicAdd(&cur[jl], 1) : gadd(&gc[bin_slot(j)], 1);
                dst.z[dest] = z[k];
                dst.vz[dest] = vzr[k];
                *(GLB u32x4 *)&dst.cold[dest] = cold[k];
                dst.tc[dest] = tcr[k];
            }
        }
        lds_barrier();
        c = run_end;
    }
}

__global__ __launch_bounds__(256) void k_sort_finalize(const Diode *__restrict__ D)
{
    const Diode &dd = D[blockIdx.x];
    for (int s = 0; s < NSP; ++s) {
        int *cc = dd.cell_cnt[s];
        for (int j = threadIdx.x; j < dd.N; j += 256) cc[j] = 0;
    }
    if (threadIdx.x == 0) {
        DiodeState *st = dd.st;
        dd.tally->resorts += 1ull;
        if (st->keep[SP_I]) dd.tally->resorts_ions_kept += 1ull;
        for (int s = 0; s < NSP; ++s) {
            if (st->keep[s]) st->flip[s] ^= 1;    // left in place: its buffer is now parity ^ 1 ^ flip
            else st->n[s] = st->n_new[s];
            st->keep[s] = 0;
        }
        st->parity ^= 1;
        st->resorts += 1u;
    }
}

// ---------------------------------------------------------------------------
// 128-bit signed integer (two's complement) for the exact double prefix scan.
// ---------------------------------------------------------------------------
struct I128 {
    unsigned long long lo;
    long long hi;
};
__device__ __forceinline__ I128 i128(long long v)
{
    I128 r;
    r.lo = (unsigned long long)v;
    r.hi = v < 0 ? -1 : 0;
    return r;
}
__device__ __forceinline__ I128 add(I128 a, I128 b)
{
    I128 r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < a.lo ? 1 : 0);
    return r;
}
__device__ __forceinline__ I128 neg(I128 a)
{
    I128 r;
    r.lo = ~a.lo + 1ull;
    r.hi = ~a.hi + (r.lo == 0ull ? 1 : 0);
    return r;
}
// a * m for 0 <= m < 2^31
__device__ __forceinline__ I128 mul_small(I128 a, unsigned m)
{
    const unsigned long long l0 = a.lo & 0xFFFFFFFFull, l1 = a.lo >> 32;
    unsigned long long p0 = l0 * m;
    unsigned long long p1 = l1 * m + (p0 >> 32);
    I128 r;
    r.lo = (p0 & 0xFFFFFFFFull) | (p1 << 32);
    r.hi = (long long)((unsigned long long)a.hi * m + (p1 >> 32));
    return r;
}
// Converts through the magnitude: hi * 2^64 + lo with a negative hi would
// cancel catastrophically for values of small magnitude.
__device__ __forceinline__ double to_double(I128 a)
{
    const bool negv = a.hi < 0;
    if (negv) a = neg(a);
    const double m = (double)(unsigned long long)a.hi * 18446744073709551616.0 + (double)a.lo;
    return negv ? -m : m;
}

__device__ void write_particle(const GBuf &b, int i, double z, float vx, float vy, float vz, uint32_t id,
                               uint32_t tc)
{
    b.z[i] = z; b.vz[i] = vz; b.tc[i] = tc;
    put_cold(&b.cold[i], vx, vy, id);
}

// Inclusive wave scans with DPP moves (ALU-latency lane exchanges, where a
// shuffle goes through the LDS crossbar and waits for it): shifts by 1, 2, 4
// and 8 lanes within each row of 16 (zero entering from the row's start),
// then the row totals broadcast from lane 15 into rows 1 and 3 and from lane
// 31 into rows 2 and 3.  Every lane of the wave must be active.
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118;
constexpr int DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143;

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, ROWS, 0xf, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, ROWS, 0xf, true);
    return ((unsigned long long)hi << 32) | lo;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ I128 dpp_i128(I128 v)
{
    I128 r;
    r.lo = dpp_u64<CTRL, ROWS>(v.lo);
    r.hi = (long long)dpp_u64<CTRL, ROWS>((unsigned long long)v.hi);
    return r;
}

__device__ __forceinline__ long long wave_incl_scan_i64(long long x)
{
    unsigned long long u = (unsigned long long)x;    // two's complement: the sums wrap as int64's do
    u += dpp_u64<DPP_ROW_SHR1, 0xf>(u);
    u += dpp_u64<DPP_ROW_SHR2, 0xf>(u);
    u += dpp_u64<DPP_ROW_SHR4, 0xf>(u);
    u += dpp_u64<DPP_ROW_SHR8, 0xf>(u);
    u += dpp_u64<DPP_ROW_BCAST15, 0xa>(u);
    u += dpp_u64<DPP_ROW_BCAST31, 0xc>(u);
    return (long long)u;
}

__device__ __forceinline__ I128 wave_incl_scan_i128(I128 x)
{
    x = add(x, dpp_i128<DPP_ROW_SHR1, 0xf>(x));
    x = add(x, dpp_i128<DPP_ROW_SHR2, 0xf>(x));
    x = add(x, dpp_i128<DPP_ROW_SHR4, 0xf>(x));
    x = add(x, dpp_i128<DPP_ROW_SHR8, 0xf>(x));
    x = add(x, dpp_i128<DPP_ROW_BCAST15, 0xa>(x));
    x = add(x, dpp_i128<DPP_ROW_BCAST31, 0xc>(x));
    return x;
}

// ---------------------------------------------------------------------------
// Sources and field.  mode 0: births, solve, field, tallies, step + 1;
// mode 1: solve and field only.
//
// Poisson: phi_{j-1} - 2 phi_j + phi_{j+1} = -alpha R_j (j = 1..N-1),
// phi_0 = 0, phi_N = V, R = H_I - H_P - H_E.  With S1_j = sum_{k=1..j} R_k and
// T_j = sum_{m=1..j-1} S1_m, both exact integers (64 and 128 bit),
// phi_j = V j / N + alpha (j T_N - N T_j) / N: the direct solution of the
// constant-coefficient Dirichlet system, rounded once at the end.
// ---------------------------------------------------------------------------
// Block scans of the per-thread totals of the first NWV waves (the other
// waves pass zeros and only take part in the barriers), for the field kernels
// whose threads each walk consecutive nodes serially in registers.
template <int NWV>
__device__ __forceinline__ long long block_scan_excl_i64(long long v, long long *sh, long long &total)
{
    const int lane = lane_id(), w = threadIdx.x >> 6;
    long long incl = 0;
    if (w < NWV) {
        incl = wave_incl_scan_i64(v);
        if (lane == 63) sh[w] = incl;
    }
    __syncthreads();
    long long off = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < NWV; ++q) {
        const long long t = sh[q];
        if (q < w) off += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return off + incl - v;
}

template <int NWV>
__device__ __forceinline__ I128 block_scan_excl_i128(I128 v, I128 *sh, I128 &total)
{
    const int lane = lane_id(), w = threadIdx.x >> 6;
    I128 incl = i128(0);
    if (w < NWV) {
        incl = wave_incl_scan_i128(v);
        if (lane == 63) sh[w] = incl;
    }
    __syncthreads();
    I128 off = i128(0), tot = i128(0);
#pragma unroll
    for (int q = 0; q < NWV; ++q) {
        const I128 t = sh[q];
        if (q < w) off = add(off, t);
        tot = add(tot, t);
    }
    __syncthreads();
    total = tot;
    return add(off, add(incl, neg(v)));
}

// ---------------------------------------------------------------------------
// Sources and field of a step in one kernel per step.
//
// Grid (tiles + 1, diodes).  Block 0 of a diode writes the newborn records
// (and works off any rare items the particle kernel spilled to the global
// lists, normally none; the other blocks wait for its flag before they read
// the counters those items change).  Block t + 1 takes tile t of the nodes:
// it works out the positions of the step's newborns itself (the same
// counter-based draws, so every block finds the same ones) and adds their
// charge and deposits, solves for the potential with exact integer prefix
// sums and writes phi, E and the node bookkeeping of its tile.  Block T + 1,
// dispatched last, applies the step's tallies, clears the tally copies and
// advances the counters once every other block of the diode has read them
// and the record block has written its tallies (a counter they bump), while
// the tiles solve.  Every wait is on blocks of the same diode dispatched
// earlier.
//
//   k_field_step   (N + 1 <= FUSED_MAX_NODES) tiles of TILE nodes; every tile
//                  block stages the charge of every node in LDS and runs the
//                  double prefix scans over all of them: phi exactly as
//                  defined, rounded once.
//   k_field_tiles  (larger grids) tiles of BIG_TILE nodes; a tile block
//                  publishes its aggregates (A_t = sum of its charge, B_t =
//                  sum over its interior nodes of the in-tile inclusive
//                  prefix, n_t interior nodes) with a flag and combines the
//                  aggregates of the tiles before it: P_t = sum_{u<t} A_u is
//                  S1 before the tile, Q_t = sum_{u<t} (n_u P_u + B_u) is T
//                  before it.  T_N needs every tile, so the tiles write
//                  phi'_j = V j / N - alpha T_j and E' from phi'; the
//                  last tile (the writer) has T_N and stores the correction
//                  phi_j = phi'_j + j c, c = alpha T_N / N, which shifts every
//                  node's E by -c / dz.  The particle kernel adds that shift
//                  to the E it gathers, the host adds both to what it reads.
// ---------------------------------------------------------------------------
constexpr int TILE = 512;                 // nodes per tile block of k_field_step
// Every node's charge staged in each block's LDS.  Above 2049 nodes the tiles'
// look-back costs less than every block scanning the whole grid (4097 nodes:
// 60.6 against 62.8 us per step); at 2049 the whole-grid scans still win in
// batches (32 diodes: 145.8 against 146.9 us per step).
constexpr int FUSED_MAX_NODES = 2049;
// nodes per tile block of k_field_tiles (one per thread of its first half:
// the per-node work of a tile runs on one CU, so smaller tiles spread it)
constexpr int BIG_TILE = FIELD_BIG_TILE;
static_assert(2 * BIG_TILE <= FT && BIG_TILE % 64 == 0, "one thread per node of a tile, whole waves, and as many waves again for the node bookkeeping");
constexpr int MAX_TILES = 32768 / BIG_TILE;    // N <= 32767: the earlier tiles fit one wave
static_assert(MAX_TILES <= 64, "one lane per earlier tile");

struct BirthPlan {
    int q, R, ne;              // ionisation events, replenished pairs, emitted electrons
    int bP, bE, bI;            // first free slot per species
    int okP, okE, okI;         // births that fit per species
    uint32_t id0;              // first newborn id
    int sorted;                // ionisation events taken in parent-id order (keys)
};

// A newborn's charge into R for the nodes [r0, r1) (interior nodes, ions
// positive) and its species deposit into the own tile's counts hb.
// What the plan and the newborns' charge need of the diode, copied into LDS
// by one thread at the start of a field block, while the counters are read:
// fetched where they are used, these fields would each cost a round trip to
// memory on the step's critical path (the particle kernel before has evicted
// them from the caches).
struct BirthConsts {
    double L, invdz, dt, emit_x, sig_c;
    const IzEvent *izq;
    uint32_t kseed;
    int N, replenish;
    int cap[NSP];
};

__device__ __forceinline__ void birth_consts(const Diode &dd, BirthConsts &bc)
{
    bc.L = dd.L;
    bc.invdz = dd.invdz;
    bc.dt = dd.dt;
    bc.emit_x = dd.emit_x;
    bc.sig_c = dd.sig_c;
    bc.izq = dd.izq;
    bc.kseed = dd.kseed;
    bc.N = dd.N;
    bc.replenish = dd.replenish;
#pragma unroll
    for (int s = 0; s < NSP; ++s) bc.cap[s] = dd.cap[s];
}

template <int HB>
__device__ __forceinline__ void fused_deposit(const BirthConsts &bc, long long *R, int r0, int r1,
                                              unsigned long long (*hb)[HB], int a0, int b0, int s, double z)
{
    int j;
    double f;
    cic(z, bc.invdz, bc.N, j, f);
    const unsigned long long a = fixed_right(f), l = (1ull << 32) - a;
    const long long sg = s == SP_I ? 1 : -1;
    if (j >= 1 && j >= r0 && j < r1)
        atomicAdd(reinterpret_cast<unsigned long long *>(&R[j - r0]), (unsigned long long)(sg * (long long)l));
    if (j + 1 <= bc.N - 1 && j + 1 >= r0 && j + 1 < r1)
        atomicAdd(reinterpret_cast<unsigned long long *>(&R[j + 1 - r0]), (unsigned long long)(sg * (long long)a));
    if (j >= a0 && j < b0) atomicAdd(&hb[s][j - a0], l);
    if (j + 1 >= a0 && j + 1 < b0) atomicAdd(&hb[s][j + 1 - a0], a);
}

// Index of the ionisation event of rank r (parent-id order when sorted).
__device__ __forceinline__ int iz_index(const BirthPlan &bp, const unsigned long long *keys, int r)
{
    return bp.sorted ? (int)(keys[r] & 0xFFFFull) : r;
}

// The positions of the step's newborns (ionisation products at their parent,
// thermionic electrons at z = v_z dt with v_z from the flux-weighted
// half-Maxwellian at Tc, replenished pairs at a shared uniform position),
// one thread per newborn (pair), deposited into the block's LDS: the charge
// of the nodes [r0, r1) into R, the species deposits of the own tile into
// hb.  (A thermionic electron placed beyond the anode is tallied with the
// records.)
template <int HB>
__device__ __forceinline__ void births_deposit(const BirthConsts &bc, const BirthPlan &bp, const unsigned long long *keys,
                                               uint32_t step, long long *R, int r0, int r1,
                                               unsigned long long (*hb)[HB], int a0, int b0)
{
    // one kind of newborn per wave (thermionic electrons on the first,
    // replenished pairs on the second, ionisation products on the others): a
    // wave holding several kinds would run their branches one after another
    const int q = bp.q, ne = bp.ne, w = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    if (w == 0) {
        for (int i = lane; i < bp.okE; i += 64) {
            const uint32_t idn = bp.id0 + 2u * q + i;
            const uint4 b0w = philox(step, EV_BIRTH, 0u, 0u, idn, bc.kseed);
            const float vz = (float)(bc.sig_c * sqrt(-2.0 * log(u53(b0w.z, b0w.w))));
            const double z = (double)vz * bc.dt;
            if (z < bc.L) fused_deposit<HB>(bc, R, r0, r1, hb, a0, b0, SP_E, z);
        }
    } else if (w == 1) {
        for (int r = lane; r < bp.R; r += 64) {
            const uint32_t ide = bp.id0 + 2u * q + ne + 2u * r;
            const uint4 e1 = philox(step, EV_BIRTH, 1u, 0u, ide, bc.kseed);
            const double z = bc.L * u53(e1.x, e1.y);
            if (q + r < bp.okP) fused_deposit<HB>(bc, R, r0, r1, hb, a0, b0, SP_P, z);
            if (q + r < bp.okI) fused_deposit<HB>(bc, R, r0, r1, hb, a0, b0, SP_I, z);
        }
    } else {
        for (int x = (int)threadIdx.x - 128; x < q; x += FT - 128) {
            const double z = bc.izq[iz_index(bp, keys, x)].z;
            if (x < bp.okP) fused_deposit<HB>(bc, R, r0, r1, hb, a0, b0, SP_P, z);
            if (x < bp.okI) fused_deposit<HB>(bc, R, r0, r1, hb, a0, b0, SP_I, z);
        }
    }
}

// The newborn records (positions as births_deposit, velocities, ids and
// first free flights), one thread per newborn (pair), each kind on waves of
// its own.
__device__ __forceinline__ void births_records(const Diode &dd, const BirthPlan &bp, const unsigned long long *keys,
                                               uint32_t step, int parity, const int *flip)
{
    const int q = bp.q, ne = bp.ne, w = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const GBuf bP = gbuf(dd.buf[parity ^ flip[SP_P]][SP_P]), bE = gbuf(dd.buf[parity ^ flip[SP_E]][SP_E]),
               bI = gbuf(dd.buf[parity ^ flip[SP_I]][SP_I]);
    // one kind of newborn per wave, as in births_deposit: thermionic
    // electrons on the first, replenished pairs on the second, ionisation
    // products on the others
    const int first = w == 0 ? q : w == 1 ? q + ne : 0;
    const int end = w == 0 ? q + ne : w == 1 ? q + ne + bp.R : q;
    const int stride = w < 2 ? 64 : FT - 128;
    for (int x = first + (w < 2 ? lane : (int)threadIdx.x - 128); x < end; x += stride) {
        if (x < q) {
            const int r = x;
            const IzEvent ev = dd.izq[iz_index(bp, keys, r)];
            const uint32_t ide = bp.id0 + 2u * r, idi = ide + 1u;
            if (r < bp.okP) {
                const uint4 be = philox(step, EV_BIRTH, 1u, 0u, ide, dd.kseed);
                write_particle(bP, bp.bP + r, ev.z, ev.ve[0], ev.ve[1], ev.ve[2], ide,
                               next_candidate(step, dd.lam[0], be.z, be.w));
            }
            if (r < bp.okI) {
                const uint4 bi = philox(step, EV_BIRTH, 1u, 0u, idi, dd.kseed);
                write_particle(bI, bp.bI + r, ev.z, ev.vi[0], ev.vi[1], ev.vi[2], idi,
                               next_candidate(step, dd.lam[1], bi.z, bi.w));
            }
        } else if (x < q + ne) {
            const int i = x - q;
            if (i >= bp.okE) continue;
            const uint32_t idn = bp.id0 + 2u * q + i;
            const uint4 b0w = philox(step, EV_BIRTH, 0u, 0u, idn, dd.kseed);
            const uint4 b1w = philox(step, EV_BIRTH, 1u, 0u, idn, dd.kseed);
            double n1, n2;
            bm32(b0w.x, b0w.y, n1, n2);
            const float vz = (float)(dd.sig_c * sqrt(-2.0 * log(u53(b0w.z, b0w.w))));
            const float vx = (float)(dd.sig_c * n1), vy = (float)(dd.sig_c * n2);
            const double z = (double)vz * dd.dt;
            const uint32_t tc = next_candidate(step, dd.lam[0], b1w.z, b1w.w);
            // a newborn beyond the anode is absorbed at once: a hole, tallied here
            write_particle(bE, bp.bE + i, z >= dd.L ? -1.0 : z, vx, vy, vz, idn, tc);
            if (z >= dd.L) {
                const double dvx = vx, dvy = vy;
                const double ke = 0.5 * dd.mass[SP_E] * (dvx * dvx + dvy * dvy + (double)vz * vz);
                atomicAdd(&dd.tally->abs_count[SP_E][1], 1ull);
                atomicAdd(&dd.tally->abs_energy[SP_E][1], ke);
                // complete before the block's arrival releases the tallies
                __threadfence();
            }
        } else {
            const int r = x - q - ne;
            const uint32_t ide = bp.id0 + 2u * q + ne + 2u * r, idi = ide + 1u;
            const uint4 e1 = philox(step, EV_BIRTH, 1u, 0u, ide, dd.kseed);
            const double z = dd.L * u53(e1.x, e1.y);
            double a1, a2, a3, a4;
            if (q + r < bp.okP) {
                const uint4 e0 = philox(step, EV_BIRTH, 0u, 0u, ide, dd.kseed);
                bm32(e0.x, e0.y, a1, a2);
                bm32(e0.z, e0.w, a3, a4);
                write_particle(bP, bp.bP + q + r, z, (float)(dd.sig_e0 * a1), (float)(dd.sig_e0 * a2),
                               (float)(dd.sig_e0 * a3), ide, next_candidate(step, dd.lam[0], e1.z, e1.w));
            }
            if (q + r < bp.okI) {
                const uint4 i0 = philox(step, EV_BIRTH, 0u, 0u, idi, dd.kseed);
                const uint4 i1 = philox(step, EV_BIRTH, 1u, 0u, idi, dd.kseed);
                bm32(i0.x, i0.y, a1, a2);
                bm32(i0.z, i0.w, a3, a4);
                write_particle(bI, bp.bI + q + r, z, (float)(dd.sig_i0 * a1), (float)(dd.sig_i0 * a2),
                               (float)(dd.sig_i0 * a3), idi, next_candidate(step, dd.lam[1], i1.z, i1.w));
            }
        }
    }
}

// The particle kernel's tally copies, read without clearing (the tail block
// clears them once every block has read them).
__device__ __forceinline__ RareTally read_tally_copy(const Diode &dd)
{
    static_assert(TALLY_COPIES == 64, "one copy per lane of the first wave");
    return dd.tacc[threadIdx.x & 63].t;
}

// The shared state of a field step's block.
struct FieldShared {
    RareTally rt, rs;          // the step's tallies (tail block), the spilled items' (record block)
    DiodeState s_st;           // the counters as this block read them
    BirthPlan bp;
    BirthConsts bc;
};

// The first reads of every block of a field step (mode 0): the particle
// kernel's tally copies (first wave) and the counters (second wave).
__device__ __forceinline__ RareTally field_step_reads(const Diode &dd, FieldShared &fs)
{
    const int tid = threadIdx.x;
    RareTally copy{};
    if (tid < 64) copy = read_tally_copy(dd);
    if (tid >= 64 && tid < 128) load_state(dd.st, &fs.s_st);
    if (tid == 192) birth_consts(dd, fs.bc);
    if (tid == 0) {
        rare_tally_zero(&fs.rt);
        rare_tally_zero(&fs.rs);
    }
    return copy;
}

// After field_step_reads and a barrier: the tail block folds every tally
// copy into fs.rt, the others only the ions lost; the spilled rare items are
// worked off (record block) or waited for; once a tile block or the record
// block is done with the counters it bumps st->arrive, then every block works
// out the plan of the step's births and, when the plan needs it, the
// ionisation events in parent-id order in keys.
// The roles of a field step's blocks (mode 0): block 0 writes the newborn
// records, blocks 1..T take the node tiles, block T + 1 (dispatched last)
// applies the step's tallies and advances the counters.
enum FieldRole { ROLE_RECORDS, ROLE_TILE, ROLE_TAIL };

__device__ void field_step_plan(const Diode &dd, int parity, uint32_t step, FieldRole role, RareTally copy,
                                FieldShared &fs, unsigned long long *keys)
{
    DiodeState *st = dd.st;
    const int tid = threadIdx.x;
    const bool records = role == ROLE_RECORDS;
    if (__builtin_expect(role == ROLE_TAIL, 0)) {
        fold_tally_copies(copy, &fs.rt);      // the step's totals, applied by the tail block
    } else if (tid < 64) {
        int v = copy.ion_lost;                // the others need the ions lost only
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (tid == 0) fs.rt.ion_lost = v;
    }
    if (__builtin_expect((fs.s_st.rare_n[SP_P] | fs.s_st.rare_n[SP_E] | fs.s_st.rare_n[SP_I]) != 0, 0)) {
        // items the particle kernel's queues could not hold: the record
        // block collides them (they may queue ionisations and lose ions),
        // then raises the flag the other blocks wait for
        if (records) {
            if (tid == 0)
                atomicAdd(&dd.tally->rare_spill,
                          (unsigned long long)(fs.s_st.rare_n[SP_P] + fs.s_st.rare_n[SP_E] + fs.s_st.rare_n[SP_I]));
            process_rare(dd, fs.s_st.rare_n, fs.s_st.flip, parity, step, tid, FT, &fs.rs);
            // every thread's queue entries and counters complete before the
            // flag (a barrier does not wait for other waves' global stores)
            __threadfence();
            __syncthreads();
            if (tid == 0) {
                apply_tally(dd, fs.rs);
                if (fs.rs.ion_lost) atomicAdd(&st->ion_lost, fs.rs.ion_lost);
                __hip_atomic_store(glb(&st->spill_flag), step + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else if (tid == 0) {
            while (__hip_atomic_load(glb(&st->spill_flag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != step + 1u)
                __builtin_amdgcn_s_sleep(2);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the record block's queue and counters
        }
        __syncthreads();
        if (tid >= 64 && tid < 128) load_state(st, &fs.s_st);
    }
    __syncthreads();
    if (tid == 0) {
        // this tile or record block is done with the counters and the copies
        if (role != ROLE_TAIL) __hip_atomic_fetch_add(glb(&st->arrive), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const DiodeState &S = fs.s_st;
        BirthPlan p;
        p.q = min(S.iz_count, IZQ_CAP);
        p.R = fs.bc.replenish ? S.ion_lost + fs.rt.ion_lost : 0;
        p.ne = 0;
        if (fs.bc.emit_x > 0.0) {
            const double fl = floor(fs.bc.emit_x);
            const uint4 be = philox(step, EV_EMIT, 0u, 0u, 0xFFFFFFFFu, fs.bc.kseed);
            p.ne = (int)fl + (u53(be.x, be.y) < fs.bc.emit_x - fl ? 1 : 0);
        }
        p.id0 = S.next_id;
        p.bP = S.n[SP_P];
        p.bE = S.n[SP_E];
        p.bI = S.n[SP_I];
        // births that do not fit are dropped (and flagged by the tail block)
        p.okP = min(p.q + p.R, fs.bc.cap[SP_P] - p.bP);
        p.okE = min(p.ne, fs.bc.cap[SP_E] - p.bE);
        p.okI = min(p.q + p.R, fs.bc.cap[SP_I] - p.bI);
        // the parent-id order names the ionisation products (the record
        // block) and, when some do not fit, decides which are dropped
        p.sorted = p.q > 1 && role != ROLE_TAIL && (records || p.okP < p.q || p.okI < p.q);
        fs.bp = p;
    }
    __syncthreads();
    if (__builtin_expect(fs.bp.sorted, 0)) {
        const int q = fs.bp.q;
        int np2 = 1;
        while (np2 < q) np2 <<= 1;
        for (int i = tid; i < np2; i += FT)
            keys[i] = i < q ? ((unsigned long long)fs.bc.izq[i].parent << 32) | (unsigned)i : ~0ull;
        __syncthreads();
        for (int k = 2; k <= np2; k <<= 1) {
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
                for (int i = tid; i < np2; i += FT) {
                    const int pi = i ^ jj;
                    if (pi > i) {
                        const unsigned long long u = keys[i], v = keys[pi];
                        const bool up = (i & k) == 0;
                        if ((u > v) == up) { keys[i] = v; keys[pi] = u; }
                    }
                }
                __syncthreads();
            }
        }
    }
}

// The tail block's end of a step (mode 0), once `others` blocks of the diode
// (the tiles and the record block) are done with the counters and the tally
// copies: the copies cleared, the step's tallies applied, the counters
// advanced; on a snapshot step, once the record block has also released its
// tallies (newborns placed beyond the anode), the snapshot taken.
__device__ void field_step_tail(const Diode &dd, FieldShared &fs, uint32_t step, int avg, int others)
{
    DiodeState *st = dd.st;
    const int tid = threadIdx.x;
    if (tid == 0) {
        while (__hip_atomic_load(glb(&st->arrive), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < others)
            __builtin_amdgcn_s_sleep(2);
        __hip_atomic_store(glb(&st->arrive), 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (tid < 64) dd.tacc[tid].t = RareTally{};
    if (tid == 0) {
        const BirthPlan &p = fs.bp;
        if (p.okP < p.q + p.R || p.okE < p.ne || p.okI < p.q + p.R) atomicOr(&st->err, ERR_CAPACITY);
        apply_tally(dd, fs.rt);
        st->n[SP_P] = p.bP + p.okP;
        st->n[SP_E] = p.bE + p.okE;
        st->n[SP_I] = p.bI + p.okI;
        st->next_id = p.id0 + 2u * p.q + p.ne + 2u * p.R;
        if (p.ne) atomicAdd(&dd.tally->n_emit, (unsigned long long)p.ne);
        if (p.R) atomicAdd(&dd.tally->n_repl, (unsigned long long)p.R);
        if (p.q) atomicAdd(&dd.tally->n_iz, (unsigned long long)p.q);
        st->iz_count = 0;
        st->ion_lost = 0;
        st->spill_flag = 0u;
#pragma unroll
        for (int sp = 0; sp < NSP; ++sp) st->rare_n[sp] = 0;
        st->step = step + 1u;
        if (avg) st->avg_steps += 1;
    }
    // every tally update of the block (births beyond the anode, the step's
    // totals) is complete before the snapshot reads the tallies
    __syncthreads();
    const uint32_t nstep = step + 1u;
    if (tid == 0 && dd.tally_period > 0 && nstep % (uint32_t)dd.tally_period == 0u) {
        // the record block (dispatched before this block) sets the flag
        while (__hip_atomic_load(glb(&st->rec_flag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != nstep)
            __builtin_amdgcn_s_sleep(2);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        TallySnap &sn = dd.ring[(nstep / (uint32_t)dd.tally_period) % RING];
        sn.step = nstep;
        sn.t = *dd.tally;
    }
}

// What a tile's potential and output need of the diode, copied into LDS by
// one thread at the start of a field block: read later, after the look-back's
// acquire loads (which invalidate the caches), each of these fields would
// cost a round trip to memory.
struct TileConsts {
    double V, alpha, dz;
    int N;
    double *phi, *E, *phi_sum;
    unsigned long long *H[NSP];
    long long *Hlast[NSP], *Hsum[NSP];
    uint32_t *err;
};

__device__ __forceinline__ void tile_consts(const Diode &dd, TileConsts &fc)
{
    fc.V = dd.V;
    fc.alpha = dd.alpha;
    fc.dz = dd.dz;
    fc.N = dd.N;
    fc.phi = dd.phi;
    fc.E = dd.E;
    fc.phi_sum = dd.phi_sum;
#pragma unroll
    for (int s = 0; s < NSP; ++s) {
        fc.H[s] = dd.H[s];
        fc.Hlast[s] = dd.Hlast[s];
        fc.Hsum[s] = dd.Hsum[s];
    }
    fc.err = &dd.st->err;
}

// A node's bookkeeping (node j, index i in the tile): the step's deposits
// (hb) into the last-step and summed histograms, and H cleared when `clear`
// (by whichever block may: every reader of the node's H has read it).
template <int HB>
__device__ __forceinline__ void field_node_hist(const TileConsts &fc, unsigned long long (*hb)[HB], int i, int j,
                                                int avg, bool clear)
{
#pragma unroll
    for (int s = 0; s < NSP; ++s) {
        const unsigned long long hu = hb[s][i];
        if (hu >= DEPOSIT_LIMIT) atomicOr(fc.err, ERR_RANGE);
        glb(fc.Hlast[s])[j] = (long long)hu;
        if (clear) glb(fc.H[s])[j] = 0ull;
        if (avg) glb(fc.Hsum[s])[j] += (long long)hu;
    }
}

// A node's field: E from phi on the tile and its halo (ph[k] = phi at node
// a0 - 1 + k, k = i + 1), phi (and its sum).
__device__ __forceinline__ void field_node_phi(const TileConsts &fc, const double *ph, int k, int j, int avg)
{
    const int N = fc.N;
    const double pc = ph[k];
    const double dz = fc.dz;
    double E;
    if (j == 0) E = (pc - ph[k + 1]) / dz;
    else if (j == N) E = (ph[k - 1] - pc) / dz;
    else E = (ph[k - 1] - ph[k + 1]) * (1.0 / (2.0 * dz));
    glb(fc.phi)[j] = pc;
    glb(fc.E)[j] = E;
    if (avg) glb(fc.phi_sum)[j] += pc;
}

// Every node's H of the diode cleared by one block.
__device__ __forceinline__ void clear_node_hist(const TileConsts &fc)
{
    const int nn = fc.N + 1;
    for (int x = threadIdx.x; x < NSP * nn; x += FT) {
        const int s = x / nn;
        glb(fc.H[s])[x - s * nn] = 0ull;
    }
}

__global__ __launch_bounds__(FT) void k_field_step(const Diode *__restrict__ D, int mode, int parity)
{
    __shared__ long long R[FUSED_MAX_NODES];          // the charge of every node
    __shared__ unsigned long long keys[IZQ_CAP];      // ionisation events by parent id
    __shared__ unsigned long long hb[NSP][TILE];      // the own tile's deposits per species
    __shared__ long long sh64[FW];
    __shared__ I128 sh128[FW];
    __shared__ double ph[TILE + 2];                   // phi on the own tile and its halo
    __shared__ I128 tT[TILE + 2];                     // T_j on the own tile and its halo
    __shared__ FieldShared fs;
    __shared__ TileConsts fc;
    __shared__ int s_avg, s_last;
    const Diode &dd = D[blockIdx.y];
    DiodeState *st = dd.st;
    const int N = dd.N, nn = N + 1;
    const int T = (nn + TILE - 1) / TILE;
    if ((int)blockIdx.x > T + 1 || ((blockIdx.x == 0 || (int)blockIdx.x == T + 1) && mode != 0)) return;
    const FieldRole role = blockIdx.x == 0 ? ROLE_RECORDS : (int)blockIdx.x == T + 1 ? ROLE_TAIL : ROLE_TILE;
    const bool records = role == ROLE_RECORDS, tile = role == ROLE_TILE;
    const int t = (int)blockIdx.x - 1;                // the tile of the tile blocks
    const int a0 = t * TILE, b0 = min(nn, a0 + TILE);
    const int tid = threadIdx.x;

    // the counters and the particle kernel's tally copies; tile blocks load
    // every node's charge and their own tile's deposits meanwhile
    RareTally copy{};
    if (mode == 0) copy = field_step_reads(dd, fs);
    if (tid == 128) tile_consts(dd, fc);
    // whether the step is averaged (the host sets avg_on between steps)
    if (tid == 1) s_avg = __hip_atomic_load(glb(&st->avg_on), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tile) {
        for (int j = tid; j < nn; j += FT) {
            long long r = 0;
            if (j >= 1 && j <= N - 1)
                r = (long long)(glb(dd.H[SP_I])[j] - glb(dd.H[SP_P])[j] - glb(dd.H[SP_E])[j]);
            R[j] = r;
        }
        for (int i = tid; i < b0 - a0; i += FT) {
#pragma unroll
            for (int s = 0; s < NSP; ++s) hb[s][i] = glb(dd.H[s])[a0 + i];
        }
    }
    const uint32_t step = mode == 0 ? (uint32_t)uni((int)st->step) : 0u;
    __syncthreads();
    const int avg = uni(s_avg);
    if (mode == 0) {
        field_step_plan(dd, parity, step, role, copy, fs, keys);
        if (__builtin_expect(records, 0)) {
            // the newborns' records and tallies; the flag releases the
            // tallies to the tail block, which waits for them only when the
            // step takes a snapshot
            births_records(dd, fs.bp, keys, step, parity, fs.s_st.flip);
            __syncthreads();
            if (tid == 0) __hip_atomic_store(glb(&st->rec_flag), step + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        if (__builtin_expect(role == ROLE_TAIL, 0)) {
            // the tiles and the record block: the step's tallies, counters and
            // snapshot; every tile block reads every node's H before it
            // arrives, so the grid's H is cleared here, after the arrivals
            field_step_tail(dd, fs, step, avg, T + 1);
            clear_node_hist(fc);
            return;
        }
        births_deposit<TILE>(fs.bc, fs.bp, keys, step, R, 0, nn, hb, a0, b0);
        __syncthreads();
    } else {
        // refield (no tail block): the last tile block to arrive, once every
        // tile block has read every node's H, clears it
        if (tid == 0)
            s_last = __hip_atomic_fetch_add(glb(&st->arrive), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == T - 1;
        __syncthreads();
        if (s_last) {
            clear_node_hist(fc);
            if (tid == 0) __hip_atomic_store(glb(&st->arrive), 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // phi_j = V j / N + alpha (j T_N - N T_j) / N with the exact sums
    // S1_j = sum_{k<=j} R_k and T_j = sum_{m=1..j-1} S1_m.  The sums run on
    // the first SCAN_WAVES waves, each thread walking `per` consecutive nodes
    // serially (serial adds cost less than wave-wide steps of more waves);
    // the T_j of the own tile and its halo go to LDS, and the potential is
    // then worked out one node per thread.
    constexpr int SCAN_WAVES = 8;
    const int per = (nn + SCAN_WAVES * 64 - 1) / (SCAN_WAVES * 64);
    const int j0 = tid < SCAN_WAVES * 64 ? tid * per : nn, j1 = min(nn, j0 + per);
    long long loc = 0;
    for (int j = j0; j < j1; ++j) loc += R[j];
    long long tot;
    const long long s1off = block_scan_excl_i64<SCAN_WAVES>(loc, sh64, tot);
    I128 tl = i128(0);
    {
        long long S1 = s1off;
        for (int j = j0; j < j1; ++j) {
            S1 += R[j];
            if (j >= 1 && j <= N - 1) tl = add(tl, i128(S1));
        }
    }
    I128 T_N;
    I128 Tacc = block_scan_excl_i128<SCAN_WAVES>(tl, sh128, T_N);
    if (j1 > a0 - 1 && j0 <= b0) {
        long long S1 = s1off;
        for (int j = j0; j < j1; ++j) {
            S1 += R[j];
            if (j >= a0 - 1 && j <= b0) tT[j - a0 + 1] = Tacc;
            if (j >= 1 && j <= N - 1) Tacc = add(Tacc, i128(S1));
        }
    }
    __syncthreads();
    const double alpha_n = fc.alpha / (double)N;
    for (int k = tid; k < b0 - a0 + 2; k += FT) {
        const int j = a0 - 1 + k;
        if (j < 0 || j > N) continue;
        double v = 0.0;
        if (j == N) v = fc.V;
        else if (j >= 1) {
            const I128 x = add(mul_small(T_N, (unsigned)j), neg(mul_small(tT[k], (unsigned)N)));
            v = fc.V * (double)j / (double)N + alpha_n * to_double(x);
        }
        ph[k] = v;
    }
    __syncthreads();
    // the own tile's field and potential on the first waves, its node
    // bookkeeping on the last ones
    static_assert(FT >= 2 * TILE, "separate waves for the field and the bookkeeping");
    if (tid < TILE) {
        if (a0 + tid < b0) field_node_phi(fc, ph, tid + 1, a0 + tid, avg);
    } else if (tid >= FT - TILE) {
        const int i = tid - (FT - TILE);
        if (a0 + i < b0) field_node_hist<TILE>(fc, hb, i, a0 + i, avg, false);
    }
}

// phi' at node j (see k_field_tiles) from the exact T_j.
__device__ __forceinline__ double phi_prime(const TileConsts &fc, int j, const I128 &Tj)
{
    if (j <= 0) return 0.0;
    return fc.V * (double)j / (double)fc.N - fc.alpha * to_double(Tj);
}

__global__ __launch_bounds__(FT) void k_field_tiles(const Diode *__restrict__ D, int mode, int parity)
{
    __shared__ long long R[BIG_TILE];                 // the own tile's charge
    __shared__ unsigned long long keys[IZQ_CAP];      // ionisation events by parent id
    __shared__ unsigned long long hb[NSP][BIG_TILE];  // the own tile's deposits per species
    __shared__ long long w_A[BIG_TILE / 64];          // per wave of the tile: sum of R,
    __shared__ I128 w_C[BIG_TILE / 64];               //   sum of the wave-local S1 over interior nodes,
    __shared__ int w_n[BIG_TILE / 64];                //   interior nodes
    __shared__ double ph[BIG_TILE + 2];               // phi' on the own tile and its halo
    __shared__ FieldShared fs;
    __shared__ long long s_P;
    __shared__ I128 s_Q, s_B;                         // S1, T before the tile; the tile's B
    __shared__ long long s_Pw[BIG_TILE / 64];         // per wave of the tile: charge of the earlier waves,
    __shared__ I128 s_Qw[BIG_TILE / 64];              //   their sum of S1 over interior nodes
    __shared__ uint32_t s_epoch;
    __shared__ int s_avg;
    __shared__ TileConsts fc;
    const Diode &dd = D[blockIdx.y];
    DiodeState *st = dd.st;
    const int N = dd.N, nn = N + 1;
    const int T = (nn + BIG_TILE - 1) / BIG_TILE;
    if ((int)blockIdx.x > T + 1 || ((blockIdx.x == 0 || (int)blockIdx.x == T + 1) && mode != 0)) return;
    const FieldRole role = blockIdx.x == 0 ? ROLE_RECORDS : (int)blockIdx.x == T + 1 ? ROLE_TAIL : ROLE_TILE;
    const bool records = role == ROLE_RECORDS, tile = role == ROLE_TILE;
    const int t = (int)blockIdx.x - 1;                // the tile of the tile blocks
    const bool writer = t == T - 1;                   // the last tile: T_N
    const int a0 = t * BIG_TILE, b0 = min(nn, a0 + BIG_TILE);
    const int tid = threadIdx.x;
    const int j = a0 + tid;                           // this thread's node

    RareTally copy{};
    if (mode == 0) copy = field_step_reads(dd, fs);
    // the launch's epoch and whether the step is averaged (the host sets
    // avg_on between steps), read with the counters at the start
    if (tid == 0) s_epoch = __hip_atomic_load(glb(&st->field_epoch), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 1) s_avg = __hip_atomic_load(glb(&st->avg_on), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 128) tile_consts(dd, fc);
    if (tile) {
        long long r = 0;
        if (j < b0) {
            unsigned long long h[NSP];
#pragma unroll
            for (int s = 0; s < NSP; ++s) {
                h[s] = glb(dd.H[s])[j];
                hb[s][tid] = h[s];
            }
            if (j >= 1 && j <= N - 1) r = (long long)(h[SP_I] - h[SP_P] - h[SP_E]);
        }
        if (tid < BIG_TILE) R[tid] = r;
    }
    const uint32_t step = mode == 0 ? (uint32_t)uni((int)st->step) : 0u;
    __syncthreads();
    const uint32_t epoch = s_epoch;
    const int avg = uni(s_avg);
    if (mode == 0) {
        field_step_plan(dd, parity, step, role, copy, fs, keys);
        if (__builtin_expect(records, 0)) {
            // the newborns' records and tallies; the flag releases the
            // tallies to the tail block, which waits for them only when the
            // step takes a snapshot
            births_records(dd, fs.bp, keys, step, parity, fs.s_st.flip);
            __syncthreads();
            if (tid == 0) __hip_atomic_store(glb(&st->rec_flag), step + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        if (__builtin_expect(role == ROLE_TAIL, 0)) {
            // once every tile has read the counters, the copies and the
            // epoch: the step's tallies, counters and snapshot, the next epoch
            field_step_tail(dd, fs, step, avg, T + 1);
            if (tid == 0) st->field_epoch = epoch + 1u;
            return;
        }
        births_deposit<BIG_TILE>(fs.bc, fs.bp, keys, step, R, a0, b0, hb, a0, b0);
        __syncthreads();
    } else if (tid == 0 && !writer) {
        // done with the epoch: the writer advances it once every tile has read it
        __hip_atomic_fetch_add(glb(&st->arrive), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }

    // The tile's aggregates with one barrier: per wave, the inclusive prefix
    // a of the charge and the exclusive prefix c of a over the interior nodes;
    // then the first wave combines the waves' totals, one lane per wave, and
    // keeps each wave's offsets in LDS for after the look-back.  With
    // P_w the charge of the earlier waves and Q_w their sum of S1 over
    // interior nodes (sum over each earlier wave of C + n P), the in-tile
    // prefix of the charge at j is s1l = P_w + a and the in-tile exclusive
    // sum of s1l over the interior nodes before j is tl = Q_w + cnt P_w + c.
    // A = the tile's charge, B = its sum of s1l over its interior nodes.
    // The tile's nodes belong to the first TW waves; the others only take
    // part in the barriers from here on.
    constexpr int TW = BIG_TILE / 64;
    const bool interior = j >= 1 && j <= N - 1 && j < b0;
    const int lane = tid & 63, wv = tid >> 6;
    long long a = 0;
    I128 c = i128(0);
    int cw = 0;
    if (wv < TW) {
        a = wave_incl_scan_i64(R[tid]);
        const I128 ci = interior ? i128(a) : i128(0);
        c = add(wave_incl_scan_i128(ci), neg(ci));
        const unsigned long long im = __ballot(interior);
        cw = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(im >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)im, 0u));
        if (lane == 63) {
            w_A[wv] = a;
            w_C[wv] = add(c, ci);
            w_n[wv] = cw + (interior ? 1 : 0);
        }
    }
    __syncthreads();
    const int nint = max(0, min(b0, N) - max(a0, 1));   // interior nodes of the tile
    if (tid < 64) {
        // one lane per wave of the tile: P_w, Q_w as exclusive scans over the
        // waves (Q_w adds each earlier wave's C + n P), the tile's A and B as
        // the last wave's inclusive ones, published at once
        const long long aw = lane < TW ? w_A[lane] : 0;
        const I128 cl = lane < TW ? w_C[lane] : i128(0);
        const int nl = lane < TW ? w_n[lane] : 0;
        const long long ai = wave_incl_scan_i64(aw);
        const I128 term = add(cl, mul_small(i128(ai - aw), (unsigned)nl));
        const I128 bi = wave_incl_scan_i128(term);
        if (lane < TW) {
            s_Pw[lane] = ai - aw;
            s_Qw[lane] = add(bi, neg(term));
        }
        if (lane == TW - 1) {
            s_B = bi;
            FieldAgg g;
            g.A = ai;
            g.B_lo = bi.lo;
            g.B_hi = bi.hi;
            g.n = nint;
            g.pad = 0;
            dd.agg[t] = g;
            // the release store orders the aggregate before the flag
            __hip_atomic_store(glb(&dd.agg_flag[t]), epoch + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (tid < 64) {
        // the tiles before this one, one lane each: P_u = sum_{v<u} A_v, the
        // sum of S1 over tile u's interior nodes n_u P_u + B_u, and their sums
        const int u = tid;
        long long Au = 0;
        I128 Bu = i128(0);
        int nu = 0;
        // Relaxed polls, then one acquire fence for the wave: an acquire load
        // invalidates the XCD's L2 on every poll (instructions included).
        if (u < t) {
            while (__hip_atomic_load(glb(&dd.agg_flag[u]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch + 1u)
                __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (u < t) {
            const FieldAgg g = dd.agg[u];
            Au = g.A;
            Bu.lo = g.B_lo;
            Bu.hi = g.B_hi;
            nu = g.n;
        }
        const long long Pu = wave_incl_scan_i64(Au) - Au;
        const I128 incl = wave_incl_scan_i128(add(mul_small(i128(Pu), (unsigned)nu), Bu));
        if (u == 63) {
            s_P = Pu + Au;      // S1 before the tile
            s_Q = incl;         // T before the tile
        }
    }
    __syncthreads();
    const long long P = s_P;
    const I128 Q = s_Q, B = s_B;
    const I128 tl = wv < TW ? add(add(s_Qw[wv], mul_small(i128(s_Pw[wv]), (unsigned)cw)), c) : i128(0);
    // exact T_j = Q + (interior nodes of the tile before j) P + tl
    if (j < b0) {
        const int cnt = max(0, min(j, N) - max(a0, 1));
        ph[tid + 1] = phi_prime(fc, j, add(add(Q, mul_small(i128(P), (unsigned)cnt)), tl));
    }
    // halo below (a wave of its own): T_{a0-1} = Q - S1_{a0-1} if a0 - 1 is
    // interior, S1_{a0-1} = P; halo above (another): T_{b0}
    if (tid == 64 && a0 >= 1) {
        const int jm = a0 - 1;
        ph[0] = phi_prime(fc, jm, (jm >= 1 && jm <= N - 1) ? add(Q, neg(i128(P))) : Q);
    }
    if (tid == 128 && b0 <= N) ph[b0 - a0 + 1] = phi_prime(fc, b0, add(add(Q, mul_small(i128(P), (unsigned)nint)), B));
    __syncthreads();
    // the tile's field and potential on its waves, its node bookkeeping on as
    // many others (after every tile's release, whose L2 write-back would
    // otherwise take these stores too); only this block reads the tile's H,
    // so it clears it
    if (j < b0) {
        field_node_phi(fc, ph, tid + 1, j, avg);
    } else if (tid >= FT - BIG_TILE) {
        const int i = tid - (FT - BIG_TILE);
        if (a0 + i < b0) field_node_hist<BIG_TILE>(fc, hb, i, a0 + i, avg, true);
    }
    if (!writer) return;
    // the writer's tile ends at node N: T_N = Q + n P + B, slope = alpha T_N / N
    if (tid == 0) {
        const I128 TN = add(add(Q, mul_small(i128(P), (unsigned)nint)), B);
        const double slope = dd.alpha / (double)N * to_double(TN);
        st->phi_slope = slope;
        st->e_shift = -slope / dd.dz;
        if (avg) st->phi_slope_sum += slope;
    }
    if (__builtin_expect(mode != 0, 0) && tid == 0) {
        // mode 1 has no record block: the writer advances the epoch once
        // every other tile has read it
        while (__hip_atomic_load(glb(&st->arrive), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < T - 1)
            __builtin_amdgcn_s_sleep(2);
        __hip_atomic_store(glb(&st->arrive), 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st->field_epoch = epoch + 1u;
    }
}

}  // namespace pic

// ---------------------------------------------------------------------------
// Launch wrappers (host side of this translation unit).
// ---------------------------------------------------------------------------
using namespace pic;

extern "C" hipError_t picx_launch_load(const Diode *D, const long long *n_load, int nd, long long max_load,
                                       hipStream_t s)
{
    if (max_load <= 0) return hipSuccess;
    dim3 grid((unsigned)((max_load + 255) / 256), nd, 2);
    hipLaunchKernelGGL(k_load, grid, dim3(256), 0, s, D, n_load);
    return hipGetLastError();
}

// max_cells: the largest N over the diodes (row length of dens)
extern "C" hipError_t picx_launch_profile_load(const Diode *D, const double *dens, int rows, int nd, int max_cells,
                                               hipStream_t s)
{
    hipLaunchKernelGGL(k_profile_count, dim3(nd), dim3(1024), 0, s, D, dens, rows, max_cells);
    hipLaunchKernelGGL(k_profile_fill, dim3((max_cells + 3) / 4, nd, 2), dim3(256), 0, s, D,
                       rows == STATE_ROWS ? dens : nullptr, max_cells);
    hipLaunchKernelGGL(k_profile_clear, dim3(nd), dim3(256), 0, s, D);
    return hipGetLastError();
}

#define PPT_DISPATCH(PPT, ...)                                      \
    switch (PPT) {                                                  \
    case 1: { constexpr int P_ = 1; __VA_ARGS__; } break;           \
    case 2: { constexpr int P_ = 2; __VA_ARGS__; } break;           \
    case 4: { constexpr int P_ = 4; __VA_ARGS__; } break;           \
    default: { constexpr int P_ = 8; __VA_ARGS__; } break;          \
    }

extern "C" hipError_t picx_launch_particles(const Diode *D, DiodeState *S, int nd, int mode, int ppt, int grid,
                                            int parity, hipStream_t s)
{
    const size_t seg_bytes = sizeof(int) * 3 * NSP * nd;
    PPT_DISPATCH(ppt, hipLaunchKernelGGL(k_particles<P_>, dim3(grid), dim3(NT), seg_bytes, s, D, S, nd, mode, parity));
    return hipGetLastError();
}

// Kernels picx_launch_sources_field enqueues for a step (timed graphs need it).
extern "C" int picx_sources_field_kernels(int max_nodes, int mode)
{
    (void)max_nodes;
    (void)mode;
    return 1;
}

// max_nodes: the largest N + 1 over the diodes.  Up to FUSED_MAX_NODES nodes
// every tile block stages the whole grid's charge (k_field_step); above, the
// tiles combine the aggregates of the tiles before them (k_field_tiles).

extern "C" hipError_t picx_launch_sources_field(const Diode *D, DiodeState *S, int nd, int mode, int max_nodes,
                                                int parity, hipStream_t s)
{
    (void)S;
    if (max_nodes <= FUSED_MAX_NODES) {
        const int tiles = (max_nodes + TILE - 1) / TILE;
        hipLaunchKernelGGL(k_field_step, dim3(tiles + 2, nd), dim3(FT), 0, s, D, mode, parity);
    } else {
        const int tiles = (max_nodes + BIG_TILE - 1) / BIG_TILE;
        hipLaunchKernelGGL(k_field_tiles, dim3(tiles + 2, nd), dim3(FT), 0, s, D, mode, parity);
    }
    return hipGetLastError();
}

// parity: the buffer current before the re-sort
extern "C" hipError_t picx_launch_sort(const Diode *D, DiodeState *S, int nd, int ppt, int grid, int parity,
                                       hipStream_t s)
{
    PPT_DISPATCH(ppt, hipLaunchKernelGGL(k_sort_count<P_>, dim3(grid), dim3(NT), 0, s, D, S, nd, parity));
    hipLaunchKernelGGL(k_sort_scan, dim3(nd * NSP), dim3(1024), 0, s, D);
    PPT_DISPATCH(ppt, hipLaunchKernelGGL(k_sort_scatter<P_>, dim3(grid), dim3(NT), 0, s, D, S, nd, parity));
    hipLaunchKernelGGL(k_sort_finalize, dim3(nd), dim3(256), 0, s, D);
    return hipGetLastError();
}

extern "C" hipError_t picx_prepare(void)
{
    return hipFuncSetAttribute((const void *)k_phase_hist, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(PHASE_MAX_BINS * sizeof(uint32_t)));
}
