// mpr_sparse.hpp -- the compacted half-sweep for gfx950: one lane per prediction site of one
// colour, so no lane work goes to sample sites.
//
// A sweep is two launches (colour 0, then colour 1) that update the state planes in place:
// within a colour no site is a neighbour of another, so each lane reads the other plane and
// writes only its own site.  The local field sums the four neighbours in the same order as the
// fused row-window kernel ((left + right) + (up + down)), from the same stored values through
// the same functions, and the site update and its Philox counter are shared, so both paths take
// identical decisions from identical states.  The bond energy is split by bond kind: the
// colour-1 launch sums the bonds of colour-1 prediction sites, the colour-0 launch the bonds
// between colour-0 prediction sites and colour-1 samples, and the sample-sample bonds are a
// constant of the data that seeds the accumulator.
//
// A wave sweeps a group of up to 32 consecutive list waves (64 entries each) of one
// (grid, chain): the control step, the reductions and the atomics are paid once per group, and
// each iteration issues the next list wave's loads before it updates its own sites (within a
// colour no listed site is read by another, so the early loads see the values the launch
// started with).
#pragma once

#include "mpr_device.hpp"

namespace mpr {

constexpr uint32_t kNoSite = 0xFFFFFFFFu;        // list padding: the lane has no site
constexpr int kMaxGroupWaves = 32;               // list waves per group, at most
constexpr int kGroupTarget = 20480;              // groups per colour before groups grow

struct SparseArgs {
    const uint32_t* sites;     // this colour's site lists: (y << 16) | plane column, padded to 64
    const int4* waves;         // per group: (grid, chain), first entry, list waves (1 ... 32), 0
    const int32_t* lead_wave;  // per (grid, chain): its first group in this colour's list
    const GcDesc* gcs;
    const GcCtl* ctl;
    const RunCtl* run;
    void* state;               // state planes, updated in place
    double* acc;
    uint32_t* acc32;           // FP16 storage: running sums in units of 2^-24 (see kAcc32)
    const uint64_t* rk_mask;   // rank tables of the compact accumulators (see acc_rank)
    const int32_t* rk_base;
    uint8_t* dec;
    GcCtl* ictl;
    int64_t* gacc;
    const int64_t* econst;     // per (grid, chain): sample-sample bond energy, two fixed-point words
    double* trace;
    double acc_target, T_min, T_max, q, J;
    int32_t n_gc, n_waves, sweep_off;    // n_waves: groups in this colour's launch
    uint32_t key0, key1;
    // one grid and one chain: the wave's entries follow from its index, so the site loads wait
    // for no table read (the (grid, chain) record is read alongside)
    int32_t single;
    int32_t group_waves;       // list waves per group (the last group of a (grid, chain) may hold fewer)
    int64_t single_base;       // first entry of this colour's list
    int32_t single_waves;      // one grid and one chain: list waves of this colour
    int32_t pad;
};

template <class St>
__device__ __forceinline__ typename St::raw buf_load_one(Rsrc r, uint32_t off)
{
    using raw = typename St::raw;
    if constexpr (sizeof(raw) == 8) {
        const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
        return ((uint64_t)v.y << 32) | v.x;
    } else if constexpr (sizeof(raw) == 4) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
    } else {
        return (raw)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
    }
}

template <class St>
__device__ __forceinline__ void buf_store_one(Rsrc r, uint32_t off, typename St::raw v)
{
    using raw = typename St::raw;
    if constexpr (sizeof(raw) == 8) {
        u32x2_t w;
        w.x = (uint32_t)v; w.y = (uint32_t)(v >> 32);
        __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)off, 0, 0);
    } else if constexpr (sizeof(raw) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)off, 0, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, r, (int)off, 0, 0);
    }
}

// half-sweep of colour C over the listed prediction sites
template <class S, class F, int FLAGS, bool PER, int C>
__global__ __launch_bounds__(256) void k_sparse(SparseArgs a)
{
    using St = Store<S>;
    using M = Math<F>;
    using Raw = typename St::raw;
    constexpr uint32_t kRaw = (uint32_t)sizeof(Raw);
    constexpr bool FUSED = (FLAGS & F_ENERGY) != 0;   // this path sums energies in double precision
    constexpr bool ACC32 = kAcc32<S>;              // FP16 storage: 32-bit running sums
    const int lane = threadIdx.x & (kWave - 1);
    const int lblock = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int wid = __builtin_amdgcn_readfirstlane(lblock * kWavesPerBlock + (int)(threadIdx.x >> 6));
    if (wid >= a.n_waves) return;                 // whole waves leave together
    int gc, nw;
    int64_t base;
    if (a.single) {
        gc = 0;
        base = a.single_base + (int64_t)wid * a.group_waves * kWave;
        nw = min(a.group_waves, a.single_waves - wid * a.group_waves);
    } else {
        const int4 wv = a.waves[wid];
        gc = __builtin_amdgcn_readfirstlane(wv.x);
        base = wv.y;
        nw = __builtin_amdgcn_readfirstlane(wv.z);
    }
    // list entries two list waves ahead, site values one ahead
    uint32_t ent_cur = a.sites[base + lane];
    uint32_t ent_next = (nw > 1) ? a.sites[base + kWave + lane] : kNoSite;
    const GcDesc g = a.gcs[gc];
    const int64_t s_abs = a.run->base_sweep + a.sweep_off;
    const uint32_t sweep = (uint32_t)s_abs;

    // colour 0 applies the previous sweep's control step; colour 1 reads what it stored
    int acc_slot = 0;
    const GcCtl ctl = sweep_control(FUSED, C == 0, gc, g, wid == a.lead_wave[gc], lane, a.ctl, a.run,
                                    a.ictl, a.gacc, a.econst, a.trace, a.n_gc, s_abs, a.J,
                                    a.acc_target, a.T_min, a.T_max, acc_slot);
    const F q = (F)a.q;
    const F J = (F)a.J;
    const F inv_piq = (F)(1.0 / (3.14159265358979323846 * a.q));
    const F alpha = (F)ctl.alpha;
    const F kexp = (sizeof(F) == 4) ? (F)(-1.4426950408889634 / ctl.T) : (F)(-1.0 / ctl.T);

    const int H = g.H, W = g.W, pitch = g.pitch;
    const int plane_sz = H * pitch;
    const int oc = (1 - C) * plane_sz;
    const Rsrc rs = make_rsrc((Raw*)a.state + g.plane_off, 2u * (uint32_t)plane_sz * kRaw);
    const Rsrc ra = ACC32 ? make_rsrc(a.acc32 + g.site_off, (uint32_t)(H * W) * 4u)
                          : make_rsrc(a.acc + g.site_off, (uint32_t)(H * W) * 8u);

    // one listed site: its entry, position, which neighbours exist, the stored values of the
    // site and of its four neighbours in the other plane (column = grid x >> 1), and (averaging
    // sweeps) the rank-table words of its compact accumulator
    struct Site {
        uint32_t ent;
        int y, k, x, xl, xr, yu, yd;
        bool valid, el, er, eu, ed;
        Raw v, rl, rr, ru, rd;
        uint64_t rkm;
        int32_t rkb;
    };
    auto fetch = [&](uint32_t ent) __attribute__((always_inline)) -> Site {
        Site t;
        t.ent = ent;
        t.valid = ent != kNoSite;
        t.y = t.valid ? (int)(ent >> 16) : 0;
        t.k = t.valid ? (int)(ent & 0xffffu) : 0;
        t.x = 2 * t.k + ((t.y + C) & 1);
        t.xl = t.x - 1; t.xr = t.x + 1; t.yu = t.y - 1; t.yd = t.y + 1;
        t.el = t.xl >= 0; t.er = t.xr < W; t.eu = t.yu >= 0; t.ed = t.yd < H;
        if (PER) {
            t.xl = t.el ? t.xl : t.xl + W; t.xr = t.er ? t.xr : t.xr - W;
            t.yu = t.eu ? t.yu : t.yu + H; t.yd = t.ed ? t.yd : t.yd - H;
            t.el = t.er = t.eu = t.ed = true;
        }
        t.el &= t.valid; t.er &= t.valid; t.eu &= t.valid; t.ed &= t.valid;
        const uint32_t own = (uint32_t)(C * plane_sz + t.y * pitch + t.k);
        t.v = buf_load_one<St>(rs, t.valid ? own * kRaw : kBufOOB);
        t.rl = buf_load_one<St>(rs, t.el ? (uint32_t)(oc + t.y * pitch + (t.xl >> 1)) * kRaw : kBufOOB);
        t.rr = buf_load_one<St>(rs, t.er ? (uint32_t)(oc + t.y * pitch + (t.xr >> 1)) * kRaw : kBufOOB);
        t.ru = buf_load_one<St>(rs, t.eu ? (uint32_t)(oc + t.yu * pitch + (t.x >> 1)) * kRaw : kBufOOB);
        t.rd = buf_load_one<St>(rs, t.ed ? (uint32_t)(oc + t.yd * pitch + (t.x >> 1)) * kRaw : kBufOOB);
        t.rkm = 0;
        t.rkb = 0;
        if constexpr ((FLAGS & F_ACC) != 0) {
            const int64_t i = g.rk_off + (int64_t)(2 * t.y + C) * (pitch >> 6) + (t.k >> 6);
            t.rkm = a.rk_mask[i];
            t.rkb = a.rk_base[i];
        }
        return t;
    };

    int n_acc = 0;
    int64_t e_hi = 0, e_lo = 0;
    auto update = [&](const Site& t) __attribute__((always_inline)) {
        const bool is_free = t.valid & !St::sample(t.v);
        // averaging sweeps: the running sum's load goes out first, the update's arithmetic
        // hides it (a scheduling barrier keeps it there)
        uint32_t ao = kBufOOB;
        double sum = 0.0;
        uint32_t sum32 = 0;
        if constexpr ((FLAGS & F_ACC) != 0) {
            const int64_t rank = (int64_t)t.rkb + (int64_t)__popcll(t.rkm & ((1ull << (t.k & 63)) - 1ull));
            ao = is_free ? (uint32_t)rank * (ACC32 ? 4u : 8u) : kBufOOB;
            if constexpr (ACC32) sum32 = __builtin_amdgcn_raw_buffer_load_b32(ra, (int)ao, 0, 0);
            else sum = buf_load_f64(ra, ao);
            __builtin_amdgcn_sched_barrier(0);
        }
        F sl, cl, sr, cr, su, cu, sd, cd;
        M::sincos_rev(q * St::template value<F>(t.rl), sl, cl);
        M::sincos_rev(q * St::template value<F>(t.rr), sr, cr);
        M::sincos_rev(q * St::template value<F>(t.ru), su, cu);
        M::sincos_rev(q * St::template value<F>(t.rd), sd, cd);
        cl = t.el ? cl : (F)0; sl = t.el ? sl : (F)0;
        cr = t.er ? cr : (F)0; sr = t.er ? sr : (F)0;
        cu = t.eu ? cu : (F)0; su = t.eu ? su : (F)0;
        cd = t.ed ? cd : (F)0; sd = t.ed ? sd : (F)0;
        const F Cf = (cl + cr) + (cu + cd);
        const F Sf = (sl + sr) + (su + sd);

        // the pair's counter; member k & 1 takes words (x, y) or (z, w)
        const U4 r = philox10(U4{(uint32_t)(t.y * g.np + (t.k >> 1)), sweep, (uint32_t)g.chain_word, (uint32_t)C},
                              a.key0, a.key1);
        const uint32_t wa = (t.k & 1) ? r.z : r.x, wb = (t.k & 1) ? r.w : r.y;
        const SiteOut<S, F> o = hybrid_update<S, F>(St::template value<F>(t.v), is_free, Cf, Sf, q, inv_piq, J,
                                                    kexp, alpha, wa, wb);
        const Raw nv = is_free ? St::template encode<F>(o.u) : t.v;
        const uint32_t own = (uint32_t)(C * plane_sz + t.y * pitch + t.k);
        buf_store_one<St>(rs, is_free ? own * kRaw : kBufOOB, nv);

        n_acc += is_free ? ((o.dec >> 1) & 1) : 0;
        if (FLAGS & F_ENERGY) {
            F e;
            if (C == 1) {
                e = M::fma(o.c, Cf, o.s * Sf);
            } else {        // bonds to colour-1 samples only
                const bool ml = t.el & St::sample(t.rl), mr = t.er & St::sample(t.rr);
                const bool mu = t.eu & St::sample(t.ru), md = t.ed & St::sample(t.rd);
                const F Cs = ((ml ? cl : (F)0) + (mr ? cr : (F)0)) + ((mu ? cu : (F)0) + (md ? cd : (F)0));
                const F Ss = ((ml ? sl : (F)0) + (mr ? sr : (F)0)) + ((mu ? su : (F)0) + (md ? sd : (F)0));
                e = M::fma(o.c, Cs, o.s * Ss);
            }
            const Fix2 f = fixed64x2(is_free ? (double)e : 0.0);
            e_hi += f.hi;
            e_lo += f.lo;
        }
        if constexpr ((FLAGS & F_ACC) != 0) {
            if constexpr (ACC32)
                __builtin_amdgcn_raw_buffer_store_b32(sum32 + acc_units<S>(nv), ra, (int)ao, 0, 0);
            else
                buf_store_f64(ra, ao, sum + St::template value<double>(nv));
        }
        if ((FLAGS & F_DEC) && is_free) a.dec[g.site_off + (int64_t)t.y * W + t.x] = (uint8_t)o.dec;
    };

    Site cur = fetch(ent_cur);
    for (int s = 0; s < nw; ++s) {
        // (wave-uniform tests: the list holds no entries past the group's last list wave)
        const uint32_t ent_after = (s + 2 < nw) ? a.sites[base + (int64_t)(s + 2) * kWave + lane] : kNoSite;
        const Site nxt = fetch(ent_next);
        __builtin_amdgcn_sched_barrier(0);      // keeps the next list wave's loads ahead of the update
        update(cur);
        cur = nxt;
        ent_next = ent_after;
    }

    if (FUSED) {
        n_acc = wave_sum_i32(n_acc);
        e_hi = wave_sum_i64(e_hi);
        e_lo = wave_sum_i64(e_lo);
        unsigned long long* A = (unsigned long long*)(a.gacc + ((int64_t)acc_slot * a.n_gc + gc) * kAccPerGc);
        // a full block of one (grid, chain) adds once (block-uniform test)
        const int b0 = lblock * kWavesPerBlock;
        const bool whole = (b0 + kWavesPerBlock <= a.n_waves) &&
                           (a.single || a.waves[b0].x == a.waves[b0 + kWavesPerBlock - 1].x);
        if (whole) {
            __shared__ int64_t red[kWavesPerBlock][3];
            const int w = (int)(threadIdx.x >> 6);
            if (lane == 0) { red[w][0] = e_hi; red[w][1] = e_lo; red[w][2] = (int64_t)n_acc; }
            __syncthreads();
            if (threadIdx.x == 0) {
                int64_t s0 = 0, s1 = 0, s2 = 0;
                for (int i = 0; i < kWavesPerBlock; ++i) { s0 += red[i][0]; s1 += red[i][1]; s2 += red[i][2]; }
                A += (blockIdx.x & (kAccCopies - 1)) * kAccStride;
                atomicAdd(A, (unsigned long long)s0);
                atomicAdd(A + kAccWord, (unsigned long long)s1);
                atomicAdd(A + 2 * kAccWord, (unsigned long long)s2);
            }
        } else if (lane == 0) {
            A += (wid & (kAccCopies - 1)) * kAccStride;
            atomicAdd(A, (unsigned long long)e_hi);
            atomicAdd(A + kAccWord, (unsigned long long)e_lo);
            atomicAdd(A + 2 * kAccWord, (unsigned long long)(int64_t)n_acc);
        }
    }
}

}  // namespace mpr
