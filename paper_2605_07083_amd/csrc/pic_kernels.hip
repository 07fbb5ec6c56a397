// pic_kernels.hip -- gfx950 kernels of the 1D3V PIC-MCC thermionic diode.
//
// One step of every diode is three launches (plus a cell re-sort every K
// steps):
//   k_particles       gather (LDS field tile) -> leapfrog push -> electrode
//                     absorption -> null-collision MCC (compacted candidate
//                     queue) -> 64-bit fixed-point CIC deposit into an LDS
//                     window histogram flushed with global integer atomics;
//   k_sources_field   one workgroup per diode: ionisation products (ordered
//                     by parent id), thermionic emission, pair replenishment,
//                     then the exact-integer double prefix-scan Poisson
//                     solve and the field, tallies and snapshots.
// Particles are processed in chunks of 256*PPT slots; the chunk list spans all
// (diode, species) segments and is walked by a persistent grid whose
// block -> chunk map keeps consecutive chunks on one XCD.
#include "pic_internal.h"

namespace pic {

constexpr int NT = 256;            // threads per particle block
constexpr int NW = NT / 64;        // wavefronts per particle block
constexpr int WMAX = 1024;         // LDS window (nodes) of the field tile / histogram
constexpr int CQ = 512;            // LDS candidate queue per chunk
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

__device__ __forceinline__ unsigned long long fixed_right(double f)
{
#pragma clang fp contract(off)
    return (unsigned long long)(long long)rint(f * TWO32);
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
// Chunk map shared by the persistent particle and sort kernels.
// ---------------------------------------------------------------------------
struct ChunkMap {
    int nseg;
    int total;
};

__device__ void build_chunk_map(const Diode *__restrict__ D, int nd, int chunk, bool use_new,
                                int *seg_end, ChunkMap &cm)
{
    int nseg = nd * NSP;
    if (threadIdx.x < 64) {
        int carry = 0;
        for (int b0 = 0; b0 < nseg; b0 += 64) {
            int sidx = b0 + threadIdx.x;
            int c = 0;
            if (sidx < nseg) {
                const DiodeState *st = D[sidx / NSP].st;
                int n = use_new ? st->n_new[sidx % NSP] : st->n[sidx % NSP];
                c = (n + chunk - 1) / chunk;
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
    cm.total = seg_end[nseg - 1];
}

// Chunks [first, total) with stride, XCD-grouped when the grid is a multiple of 8:
// block b runs on XCD b % 8 and walks that XCD's contiguous share of chunks.
__device__ __forceinline__ void chunk_range(int total, int &first, int &end, int &stride)
{
    int G = gridDim.x, b = blockIdx.x;
    if ((G & 7) == 0) {
        int x = b & 7, l = b >> 3, per = (total + 7) >> 3;
        first = x * per + l;
        end = min(total, (x + 1) * per);
        stride = G >> 3;
    } else {
        first = b;
        end = total;
        stride = G;
    }
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

// ---------------------------------------------------------------------------
// MCC for one candidate (FP32 kinematics).  Channels are tested in the fixed
// order (e: elastic, excitation, ionisation; ion: charge exchange, elastic);
// a uniform times nu_max picks the first channel whose cumulative frequency
// exceeds it, otherwise the collision is null.
// ---------------------------------------------------------------------------
struct ChunkCounts {
    int cand;
    int coll[NCH];
};

__device__ void mcc_one(const Diode &dd, int s, const SpeciesBuf &b, int i, uint32_t step, double zn,
                        float vzn, ChunkCounts *cc)
{
    const int ion = (s == SP_I);
    float vx = b.vx[i], vy = b.vy[i], vz = vzn;
    const uint32_t id = b.id[i];
    uint4 C0 = philox(step, EV_COLL, 0u, 0u, id, dd.kseed);
    uint4 C1 = philox(step, EV_COLL, 1u, 0u, id, dd.kseed);
    uint4 C2 = philox(step, EV_COLL, 2u, 0u, id, dd.kseed);
    const float sn = dd.sig_n[ion];
    float a1, a2, a3, a4;
    bm24(C0.x, C0.y, a1, a2);
    bm24(C0.z, C0.w, a3, a4);
    const float vnx = sn * a1, vny = sn * a2, vnz = sn * a3;
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
    const uint32_t tcn = next_candidate(step, dd.lam[ion], C2.z, C2.w);
    atomicAdd(&cc->cand, 1);
    if (taken >= 0) {
        atomicAdd(&cc->coll[taken], 1);
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
                    ev.z = zn;
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
        b.vx[i] = vx;
        b.vy[i] = vy;
    }
    b.vz[i] = vz;
    b.tc[i] = tcn;
}

// ---------------------------------------------------------------------------
// Particle kernel.  mode 0: full step; mode 1: deposit only (load / refield).
// ---------------------------------------------------------------------------
template <int PPT>
__global__ __launch_bounds__(NT) void k_particles(const Diode *__restrict__ D, int nd, int mode)
{
    constexpr int CHUNK = NT * PPT;
    __shared__ int seg_end[NSP * MAX_DIODES];
    __shared__ int red[2 * NW];
    __shared__ double etile[WMAX + 2];
    __shared__ unsigned long long hist[WMAX + 2];
    __shared__ int q_idx[CQ];
    __shared__ float q_vz[CQ];
    __shared__ double q_z[CQ];
    __shared__ int q_n;
    __shared__ ChunkCounts cc;

    ChunkMap cm;
    build_chunk_map(D, nd, CHUNK, false, seg_end, cm);
    int first, end, stride;
    chunk_range(cm.total, first, end, stride);
    const int tid = threadIdx.x;

    for (int c = first; c < end; c += stride) {
        const int seg = find_seg(seg_end, cm.nseg, c);
        const int d = seg / NSP, s = seg - d * NSP;
        const int base = (c - (seg ? seg_end[seg - 1] : 0)) * CHUNK;
        const Diode &dd = D[d];
        DiodeState *st = dd.st;
        const int n = st->n[s];
        const int par = st->parity;
        const uint32_t step = st->step;
        const SpeciesBuf b = dd.buf[par][s];
        const int N = dd.N;
        const double invdz = dd.invdz;

        if (tid == 0) {
            q_n = 0;
            cc.cand = 0;
#pragma unroll
            for (int k = 0; k < NCH; ++k) cc.coll[k] = 0;
        }

        double z[PPT];
        bool alive[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            int i = base + k * NT + tid;
            z[k] = -1.0;
            if (i < n) z[k] = b.z[i];
            alive[k] = z[k] >= 0.0;
        }

        if (mode == 0) {
            float vz[PPT];
            uint32_t tc[PPT];
            int jo[PPT];
            double fo[PPT];
            int mn = 0x7fffffff, mx = -1;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                int i = base + k * NT + tid;
                if (alive[k]) {
                    vz[k] = b.vz[i];
                    tc[k] = b.tc[i];
                    cic(z[k], invdz, N, jo[k], fo[k]);
                    mn = min(mn, jo[k]);
                    mx = max(mx, jo[k]);
                }
            }
            block_minmax(mn, mx, red);
            if (mx < 0) {  // no live particle in this chunk
                __syncthreads();
                continue;
            }
            // field tile: nodes mn .. mx+1 (at most WMAX+1 of them) staged in LDS
            const int g0 = mn;
            const int gcount = min(mx + 2 - mn, WMAX + 1);
            for (int t = tid; t < gcount; t += NT) etile[t] = dd.E[g0 + t];
            __syncthreads();
            const double qmdt = dd.qmdt[s], dt = dd.dt, L = dd.L;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (!alive[k]) continue;
                const int i = base + k * NT + tid;
                double e0, e1;
                const int jl = jo[k] - g0;
                if (jl + 1 < gcount) { e0 = etile[jl]; e1 = etile[jl + 1]; }
                else { e0 = dd.E[jo[k]]; e1 = dd.E[jo[k] + 1]; }
                double Ep;
                {
#pragma clang fp contract(off)
                    Ep = (1.0 - fo[k]) * e0 + fo[k] * e1;
                }
                const float vzn = (float)((double)vz[k] + qmdt * Ep);
                const double zn = z[k] + (double)vzn * dt;
                if (zn <= 0.0 || zn >= L) {
                    // absorbing electrodes
                    const int wall = zn <= 0.0 ? 0 : 1;
                    const double vxa = b.vx[i], vya = b.vy[i], vza = vzn;
                    const double ke = 0.5 * dd.mass[s] * (vxa * vxa + vya * vya + vza * vza);
                    atomicAdd(&dd.tally->abs_count[s][wall], 1ull);
                    atomicAdd(&dd.tally->abs_energy[s][wall], ke);
                    if (s == SP_I) atomicAdd(&st->ion_lost, 1);
                    b.z[i] = -1.0;
                    alive[k] = false;
                    continue;
                }
                if (!(zn == zn)) atomicOr(&st->err, ERR_NAN);
                z[k] = zn;
                b.z[i] = zn;
                if (tc[k] == step) {
                    int q = atomicAdd(&q_n, 1);
                    if (q < CQ) { q_idx[q] = i; q_vz[q] = vzn; q_z[q] = zn; }
                    else mcc_one(dd, s, b, i, step, zn, vzn, &cc);
                } else {
                    b.vz[i] = vzn;
                }
            }
        }

        // ---- deposit: LDS window histogram of the new positions ----
        int jn[PPT];
        unsigned long long an[PPT];
        int mn = 0x7fffffff, mx = -1;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!alive[k]) continue;
            double f;
            cic(z[k], invdz, N, jn[k], f);
            an[k] = fixed_right(f);
            mn = min(mn, jn[k]);
            mx = max(mx, jn[k]);
        }
        block_minmax(mn, mx, red);
        if (mx >= 0) {
            const int h0 = mn;
            const int hcount = min(mx + 2 - mn, WMAX + 1);
            for (int t = tid; t < hcount; t += NT) hist[t] = 0ull;
            __syncthreads();
            unsigned long long *H = dd.H[s];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (!alive[k]) continue;
                const int jl = jn[k] - h0;
                const unsigned long long left = (1ull << 32) - an[k];
                if (jl + 1 < hcount) {
                    if (left) atomicAdd(&hist[jl], left);
                    if (an[k]) atomicAdd(&hist[jl + 1], an[k]);
                } else {
                    atomicAdd(&H[jn[k]], left);
                    atomicAdd(&H[jn[k] + 1], an[k]);
                }
            }
            __syncthreads();
            for (int t = tid; t < hcount; t += NT) {
                unsigned long long v = hist[t];
                if (v) atomicAdd(&H[h0 + t], v);
            }
        }

        // ---- null-collision candidates of this chunk, all lanes busy ----
        if (mode == 0) {
            __syncthreads();
            const int qn = min(q_n, CQ);
            for (int q = tid; q < qn; q += NT) mcc_one(dd, s, b, q_idx[q], step, q_z[q], q_vz[q], &cc);
            __syncthreads();
            if (tid == 0) {
                const int ion = (s == SP_I);
                if (cc.cand) atomicAdd(&dd.tally->cand[ion], (unsigned long long)cc.cand);
#pragma unroll
                for (int k = 0; k < NCH; ++k)
                    if (cc.coll[k]) atomicAdd(&dd.tally->coll[k], (unsigned long long)cc.coll[k]);
            }
        }
        __syncthreads();
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
    const SpeciesBuf b = dd.buf[0][s];
    b.z[i] = dd.L * u53(b1.x, b1.y);
    b.vx[i] = (float)(sig * n1);
    b.vy[i] = (float)(sig * n2);
    b.vz[i] = (float)(sig * n3);
    b.id[i] = id;
    uint32_t tc = next_candidate(0u, dd.lam[s == SP_I], b1.z, b1.w);
    if (tc != NEVER) tc -= 1u;
    b.tc[i] = tc;
}

// ---------------------------------------------------------------------------
// Cell re-sort: count -> scan -> scatter -> finalize (compacts holes too).
// ---------------------------------------------------------------------------
template <int PPT>
__global__ __launch_bounds__(NT) void k_sort_count(const Diode *__restrict__ D, int nd)
{
    constexpr int CHUNK = NT * PPT;
    __shared__ int seg_end[NSP * MAX_DIODES];
    __shared__ int red[2 * NW];
    __shared__ int cnt[WMAX + 2];
    ChunkMap cm;
    build_chunk_map(D, nd, CHUNK, false, seg_end, cm);
    int first, end, stride;
    chunk_range(cm.total, first, end, stride);
    const int tid = threadIdx.x;
    for (int c = first; c < end; c += stride) {
        const int seg = find_seg(seg_end, cm.nseg, c);
        const int d = seg / NSP, s = seg - d * NSP;
        const int base = (c - (seg ? seg_end[seg - 1] : 0)) * CHUNK;
        const Diode &dd = D[d];
        const int n = dd.st->n[s];
        const SpeciesBuf b = dd.buf[dd.st->parity][s];
        int j[PPT];
        bool alive[PPT];
        int mn = 0x7fffffff, mx = -1;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            int i = base + k * NT + tid;
            double z = i < n ? b.z[i] : -1.0;
            alive[k] = z >= 0.0;
            if (alive[k]) {
                double f;
                cic(z, dd.invdz, dd.N, j[k], f);
                mn = min(mn, j[k]);
                mx = max(mx, j[k]);
            }
        }
        block_minmax(mn, mx, red);
        if (mx >= 0) {
            const int w = min(mx + 1 - mn, WMAX + 1);
            for (int t = tid; t < w; t += NT) cnt[t] = 0;
            __syncthreads();
            int *cc = dd.cell_cnt[s];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (!alive[k]) continue;
                int jl = j[k] - mn;
                if (jl < w) atomicAdd(&cnt[jl], 1);
                else atomicAdd(&cc[j[k]], 1);
            }
            __syncthreads();
            for (int t = tid; t < w; t += NT)
                if (cnt[t]) atomicAdd(&cc[mn + t], cnt[t]);
        }
        __syncthreads();
    }
}

// One workgroup per (diode, species): exclusive scan of the cell counts.
__global__ __launch_bounds__(1024) void k_sort_scan(const Diode *__restrict__ D)
{
    __shared__ int part[1024];
    const int d = blockIdx.x / NSP, s = blockIdx.x % NSP;
    const Diode &dd = D[d];
    const int N = dd.N;
    int *cc = dd.cell_cnt[s];
    const int per = (N + 1023) / 1024;
    const int j0 = threadIdx.x * per;
    int local = 0;
    for (int j = j0; j < min(N, j0 + per); ++j) local += cc[j];
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
        int v = cc[j];
        cc[j] = run;
        run += v;
    }
    if (threadIdx.x == 1023) dd.st->n_new[s] = part[1023];
}

template <int PPT>
__global__ __launch_bounds__(NT) void k_sort_scatter(const Diode *__restrict__ D, int nd)
{
    constexpr int CHUNK = NT * PPT;
    __shared__ int seg_end[NSP * MAX_DIODES];
    __shared__ int red[2 * NW];
    __shared__ int cnt[WMAX + 2];
    ChunkMap cm;
    build_chunk_map(D, nd, CHUNK, false, seg_end, cm);
    int first, end, stride;
    chunk_range(cm.total, first, end, stride);
    const int tid = threadIdx.x;
    for (int c = first; c < end; c += stride) {
        const int seg = find_seg(seg_end, cm.nseg, c);
        const int d = seg / NSP, s = seg - d * NSP;
        const int base = (c - (seg ? seg_end[seg - 1] : 0)) * CHUNK;
        const Diode &dd = D[d];
        const int n = dd.st->n[s];
        const int par = dd.st->parity;
        const SpeciesBuf src = dd.buf[par][s], dst = dd.buf[par ^ 1][s];
        int j[PPT], rank[PPT];
        double z[PPT];
        bool alive[PPT];
        int mn = 0x7fffffff, mx = -1;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            int i = base + k * NT + tid;
            z[k] = i < n ? src.z[i] : -1.0;
            alive[k] = z[k] >= 0.0;
            if (alive[k]) {
                double f;
                cic(z[k], dd.invdz, dd.N, j[k], f);
                mn = min(mn, j[k]);
                mx = max(mx, j[k]);
            }
        }
        block_minmax(mn, mx, red);
        if (mx >= 0) {
            const int w = min(mx + 1 - mn, WMAX + 1);
            for (int t = tid; t < w; t += NT) cnt[t] = 0;
            __syncthreads();
            int *cur = dd.cell_cnt[s];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (!alive[k]) continue;
                int jl = j[k] - mn;
                if (jl < w) rank[k] = atomicAdd(&cnt[jl], 1);
                else rank[k] = -1 - atomicAdd(&cur[j[k]], 1);   // outlier: global slot
            }
            __syncthreads();
            for (int t = tid; t < w; t += NT) {
                int v = cnt[t];
                if (v) cnt[t] = atomicAdd(&cur[mn + t], v);
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (!alive[k]) continue;
                const int i = base + k * NT + tid;
                int dest = rank[k] >= 0 ? cnt[j[k] - mn] + rank[k] : -1 - rank[k];
                dst.z[dest] = z[k];
                dst.vz[dest] = src.vz[i];
                dst.vx[dest] = src.vx[i];
                dst.vy[dest] = src.vy[i];
                dst.id[dest] = src.id[i];
                dst.tc[dest] = src.tc[i];
            }
        }
        __syncthreads();
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
        for (int s = 0; s < NSP; ++s) dd.st->n[s] = dd.st->n_new[s];
        dd.st->parity ^= 1;
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

// ---------------------------------------------------------------------------
// Sources and field: one workgroup of 1024 threads per diode.
// mode 0: births, solve, field, tallies, step + 1; mode 1: solve and field only.
// ---------------------------------------------------------------------------
constexpr int FT = 1024;
constexpr int FW = FT / 64;

template <typename T, typename Op>
__device__ __forceinline__ T block_excl_scan(T v, T *sh, Op op, T zero, T &total)
{
    // Hillis-Steele over the 1024 thread values in LDS
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < FT; o <<= 1) {
        T t = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : zero;
        __syncthreads();
        if (threadIdx.x >= (unsigned)o) sh[threadIdx.x] = op(sh[threadIdx.x], t);
        __syncthreads();
    }
    T incl = sh[threadIdx.x];
    total = sh[FT - 1];
    __syncthreads();
    T excl = threadIdx.x ? sh[threadIdx.x - 1] : zero;
    __syncthreads();
    (void)incl;
    return excl;
}

struct AddI64 {
    __device__ long long operator()(long long a, long long b) const { return a + b; }
};
struct AddI128 {
    __device__ I128 operator()(I128 a, I128 b) const { return add(a, b); }
};

__device__ __forceinline__ void deposit_global(const Diode &dd, int s, double z)
{
    int j;
    double f;
    cic(z, dd.invdz, dd.N, j, f);
    unsigned long long a = fixed_right(f);
    atomicAdd(&dd.H[s][j], (1ull << 32) - a);
    atomicAdd(&dd.H[s][j + 1], a);
}

__device__ void write_particle(const SpeciesBuf &b, int i, double z, float vx, float vy, float vz, uint32_t id,
                               uint32_t tc)
{
    b.z[i] = z; b.vx[i] = vx; b.vy[i] = vy; b.vz[i] = vz; b.id[i] = id; b.tc[i] = tc;
}

__global__ __launch_bounds__(FT) void k_sources_field(const Diode *__restrict__ D, int mode)
{
    const Diode &dd = D[blockIdx.x];
    DiodeState *st = dd.st;
    const int tid = threadIdx.x;
    __shared__ unsigned long long keys[IZQ_CAP];
    __shared__ long long sh64[FT];
    __shared__ I128 sh128[FT];
    __shared__ double phl[FT], phr[FT];
    __shared__ int s_ne, s_q, s_R, s_bP, s_bE, s_bI, s_okP, s_okE, s_okI;
    __shared__ uint32_t s_id0, s_step;

    if (mode == 0) {
        if (tid == 0) {
            const uint32_t step = st->step;
            const int q = min(st->iz_count, IZQ_CAP);
            const int R = dd.replenish ? st->ion_lost : 0;
            int ne = 0;
            if (dd.emit_x > 0.0) {
                const double fl = floor(dd.emit_x);
                uint4 be = philox(step, EV_EMIT, 0u, 0u, 0xFFFFFFFFu, dd.kseed);
                ne = (int)fl + (u53(be.x, be.y) < dd.emit_x - fl ? 1 : 0);
            }
            s_q = q; s_R = R; s_ne = ne; s_step = step; s_id0 = st->next_id;
            s_bP = st->n[SP_P]; s_bE = st->n[SP_E]; s_bI = st->n[SP_I];
            // capacity: births that do not fit are dropped and flagged
            s_okP = min(q + R, dd.cap[SP_P] - s_bP);
            s_okE = min(ne, dd.cap[SP_E] - s_bE);
            s_okI = min(q + R, dd.cap[SP_I] - s_bI);
            if (s_okP < q + R || s_okE < ne || s_okI < q + R) atomicOr(&st->err, ERR_CAPACITY);
        }
        __syncthreads();
        const int q = s_q, R = s_R, ne = s_ne;
        const uint32_t step = s_step, id0 = s_id0;
        const int par = st->parity;
        const SpeciesBuf bP = dd.buf[par][SP_P], bE = dd.buf[par][SP_E], bI = dd.buf[par][SP_I];

        // ionisation products ordered by parent id (bitonic sort in LDS)
        if (q > 0) {
            int np2 = 1;
            while (np2 < q) np2 <<= 1;
            for (int t = tid; t < np2; t += FT)
                keys[t] = t < q ? ((unsigned long long)dd.izq[t].parent << 32) | (unsigned)t : ~0ull;
            __syncthreads();
            for (int k = 2; k <= np2; k <<= 1) {
                for (int jj = k >> 1; jj > 0; jj >>= 1) {
                    for (int t = tid; t < np2; t += FT) {
                        int p = t ^ jj;
                        if (p > t) {
                            unsigned long long a = keys[t], bb = keys[p];
                            bool up = (t & k) == 0;
                            if ((a > bb) == up) { keys[t] = bb; keys[p] = a; }
                        }
                    }
                    __syncthreads();
                }
            }
            const double lam_e = dd.lam[0], lam_i = dd.lam[1];
            for (int r = tid; r < q; r += FT) {
                const IzEvent ev = dd.izq[(int)(keys[r] & 0xFFFFFFFFull)];
                const uint32_t ide = id0 + 2u * r, idi = ide + 1u;
                uint4 be = philox(step, EV_BIRTH, 1u, 0u, ide, dd.kseed);
                uint4 bi = philox(step, EV_BIRTH, 1u, 0u, idi, dd.kseed);
                if (r < s_okP) {
                    write_particle(bP, s_bP + r, ev.z, ev.ve[0], ev.ve[1], ev.ve[2], ide,
                                   next_candidate(step, lam_e, be.z, be.w));
                    deposit_global(dd, SP_P, ev.z);
                }
                if (r < s_okI) {
                    write_particle(bI, s_bI + r, ev.z, ev.vi[0], ev.vi[1], ev.vi[2], idi,
                                   next_candidate(step, lam_i, bi.z, bi.w));
                    deposit_global(dd, SP_I, ev.z);
                }
            }
        }
        // thermionic emission: flux-weighted half-Maxwellian at Tc, z = v_z dt
        for (int i = tid; i < ne; i += FT) {
            const uint32_t idn = id0 + 2u * q + i;
            uint4 b0 = philox(step, EV_BIRTH, 0u, 0u, idn, dd.kseed);
            uint4 b1 = philox(step, EV_BIRTH, 1u, 0u, idn, dd.kseed);
            double n1, n2;
            bm32(b0.x, b0.y, n1, n2);
            const float vz = (float)(dd.sig_c * sqrt(-2.0 * log(u53(b0.z, b0.w))));
            const float vx = (float)(dd.sig_c * n1), vy = (float)(dd.sig_c * n2);
            const double z = (double)vz * dd.dt;
            const uint32_t tc = next_candidate(step, dd.lam[0], b1.z, b1.w);
            if (i < s_okE) {
                if (z >= dd.L) {
                    const double ke = 0.5 * dd.mass[SP_E] *
                                      ((double)vx * vx + (double)vy * vy + (double)vz * vz);
                    atomicAdd(&dd.tally->abs_count[SP_E][1], 1ull);
                    atomicAdd(&dd.tally->abs_energy[SP_E][1], ke);
                    write_particle(bE, s_bE + i, -1.0, vx, vy, vz, idn, tc);
                } else {
                    write_particle(bE, s_bE + i, z, vx, vy, vz, idn, tc);
                    deposit_global(dd, SP_E, z);
                }
            }
        }
        // pair replenishment: one e-ion pair per ion lost this step, shared
        // uniform position, Maxwellian at the initial temperatures
        for (int r = tid; r < R; r += FT) {
            const uint32_t ide = id0 + 2u * q + ne + 2u * r, idi = ide + 1u;
            uint4 e0 = philox(step, EV_BIRTH, 0u, 0u, ide, dd.kseed);
            uint4 e1 = philox(step, EV_BIRTH, 1u, 0u, ide, dd.kseed);
            uint4 i0 = philox(step, EV_BIRTH, 0u, 0u, idi, dd.kseed);
            uint4 i1 = philox(step, EV_BIRTH, 1u, 0u, idi, dd.kseed);
            const double z = dd.L * u53(e1.x, e1.y);
            double a1, a2, a3, a4;
            bm32(e0.x, e0.y, a1, a2);
            bm32(e0.z, e0.w, a3, a4);
            if (q + r < s_okP) {
                write_particle(bP, s_bP + q + r, z, (float)(dd.sig_e0 * a1), (float)(dd.sig_e0 * a2),
                               (float)(dd.sig_e0 * a3), ide, next_candidate(step, dd.lam[0], e1.z, e1.w));
                deposit_global(dd, SP_P, z);
            }
            bm32(i0.x, i0.y, a1, a2);
            bm32(i0.z, i0.w, a3, a4);
            if (q + r < s_okI) {
                write_particle(bI, s_bI + q + r, z, (float)(dd.sig_i0 * a1), (float)(dd.sig_i0 * a2),
                               (float)(dd.sig_i0 * a3), idi, next_candidate(step, dd.lam[1], i1.z, i1.w));
                deposit_global(dd, SP_I, z);
            }
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) {
            st->n[SP_P] = s_bP + s_okP;
            st->n[SP_E] = s_bE + s_okE;
            st->n[SP_I] = s_bI + s_okI;
            st->next_id = id0 + 2u * q + ne + 2u * R;
            dd.tally->n_emit += ne;
            dd.tally->n_repl += R;
            dd.tally->n_iz += q;
            st->iz_count = 0;
            st->ion_lost = 0;
        }
    }
    __syncthreads();

    // ---- Poisson: phi_{j-1} - 2 phi_j + phi_{j+1} = -alpha R_j, phi_0 = 0, phi_N = V.
    // With S1_j = sum_{k=1..j} R_k and T_j = sum_{m=1..j-1} S1_m (exact integers),
    // phi_j = V j / N + alpha (j T_N - N T_j) / N.
    const int N = dd.N;
    const int nn = N + 1;
    const int per = (nn + FT - 1) / FT;
    const int j0 = tid * per;
    const int j1 = min(nn, j0 + per);      // nodes [j0, j1)
    constexpr int MAXPER = 32;              // N <= 32767
    long long Rl[MAXPER];
    long long s1loc = 0;
    for (int q = 0; q < per; ++q) {
        const int j = j0 + q;
        long long v = 0;
        if (j < j1 && j >= 1 && j <= N - 1)
            v = (long long)(dd.H[SP_I][j] - dd.H[SP_P][j] - dd.H[SP_E][j]);
        Rl[q] = v;
        s1loc += v;
    }
    long long tot64;
    long long s1off = block_excl_scan<long long>(s1loc, sh64, AddI64(), 0ll, tot64);
    // S1 at each own node (inclusive), and the local sums of S1 over m < j
    I128 tloc = i128(0);
    {
        long long run = s1off;
        for (int q = 0; q < per; ++q) {
            const int j = j0 + q;
            if (j >= j1) break;
            run += Rl[q];
            Rl[q] = run;                                  // now S1_j
            if (j >= 1 && j <= N - 1) tloc = add(tloc, i128(run));
        }
    }
    I128 T_N;
    I128 toff = block_excl_scan<I128>(tloc, sh128, AddI128(), i128(0), T_N);
    const double alpha_n = dd.alpha / (double)N;
    double phi_loc[MAXPER];
    {
        I128 T = toff;                                     // T_{j0} = sum_{m < j0} S1_m
        for (int q = 0; q < per; ++q) {
            const int j = j0 + q;
            if (j >= j1) break;
            double phi;
            if (j == 0) phi = 0.0;
            else if (j == N) phi = dd.V;
            else {
                I128 x = add(mul_small(T_N, (unsigned)j), neg(mul_small(T, (unsigned)N)));
                phi = dd.V * (double)j / (double)N + alpha_n * to_double(x);
            }
            phi_loc[q] = phi;
            if (j >= 1 && j <= N - 1) T = add(T, i128(Rl[q]));
        }
    }
    // neighbours across thread boundaries
    phl[tid] = j0 < j1 ? phi_loc[0] : 0.0;
    phr[tid] = j0 < j1 ? phi_loc[j1 - j0 - 1] : 0.0;
    __syncthreads();
    const double inv2dz = 1.0 / (2.0 * dd.dz);
    for (int q = 0; q < per; ++q) {
        const int j = j0 + q;
        if (j >= j1) break;
        const double ph = phi_loc[q];
        double pm = q > 0 ? phi_loc[q - 1] : (tid > 0 ? phr[tid - 1] : 0.0);
        double pp = j + 1 < j1 ? phi_loc[q + 1] : (tid + 1 < FT ? phl[tid + 1] : 0.0);
        double E;
        if (j == 0) E = (ph - pp) / dd.dz;
        else if (j == N) E = (pm - ph) / dd.dz;
        else E = (pm - pp) * inv2dz;
        dd.phi[j] = ph;
        dd.E[j] = E;
    }
    // keep the last deposit, clear the accumulators, time averages
    const int avg = st->avg_on;
    for (int j = tid; j < nn; j += FT) {
        for (int s = 0; s < NSP; ++s) {
            const long long h = (long long)dd.H[s][j];
            dd.Hlast[s][j] = h;
            dd.H[s][j] = 0ull;
            if (avg) dd.Hsum[s][j] += h;
        }
        if (avg) dd.phi_sum[j] += dd.phi[j];
    }
    __syncthreads();
    if (mode == 0 && tid == 0) {
        const uint32_t nstep = st->step + 1u;
        st->step = nstep;
        if (avg) st->avg_steps += 1;
        if (dd.tally_period > 0 && nstep % (uint32_t)dd.tally_period == 0u) {
            TallySnap &sn = dd.ring[(nstep / (uint32_t)dd.tally_period) % RING];
            sn.step = nstep;
            sn.t = *dd.tally;
        }
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

#define PPT_DISPATCH(PPT, ...)                                      \
    switch (PPT) {                                                  \
    case 1: { constexpr int P_ = 1; __VA_ARGS__; } break;           \
    case 2: { constexpr int P_ = 2; __VA_ARGS__; } break;           \
    case 4: { constexpr int P_ = 4; __VA_ARGS__; } break;           \
    default: { constexpr int P_ = 8; __VA_ARGS__; } break;          \
    }

extern "C" hipError_t picx_launch_particles(const Diode *D, int nd, int mode, int ppt, int grid, hipStream_t s)
{
    PPT_DISPATCH(ppt, hipLaunchKernelGGL(k_particles<P_>, dim3(grid), dim3(NT), 0, s, D, nd, mode));
    return hipGetLastError();
}

extern "C" hipError_t picx_launch_sources_field(const Diode *D, int nd, int mode, hipStream_t s)
{
    hipLaunchKernelGGL(k_sources_field, dim3(nd), dim3(FT), 0, s, D, mode);
    return hipGetLastError();
}

extern "C" hipError_t picx_launch_sort(const Diode *D, int nd, int ppt, int grid, hipStream_t s)
{
    PPT_DISPATCH(ppt, hipLaunchKernelGGL(k_sort_count<P_>, dim3(grid), dim3(NT), 0, s, D, nd));
    hipLaunchKernelGGL(k_sort_scan, dim3(nd * NSP), dim3(1024), 0, s, D);
    PPT_DISPATCH(ppt, hipLaunchKernelGGL(k_sort_scatter<P_>, dim3(grid), dim3(NT), 0, s, D, nd));
    hipLaunchKernelGGL(k_sort_finalize, dim3(nd), dim3(256), 0, s, D);
    return hipGetLastError();
}
