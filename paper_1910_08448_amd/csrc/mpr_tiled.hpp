// mpr_tiled.hpp -- the LDS-tiled checkerboard sweep for gfx950: one launch per sweep, one
// block per tile of TY rows x kTileCols plane columns of both colour planes of one (grid,
// chain).
//
// A block stages its tile with a halo in LDS: the colour-1 plane two rows / columns around it
// (old values), the colour-0 plane one around it.  It updates the colour-0 prediction sites of
// the tile and of the one-site ring around it (the ring repeats the neighbouring tiles' colour-0
// updates bit for bit: same inputs, same counters), then, after one block barrier, the colour-1
// prediction sites of the tile from the new colour-0 values.  Only prediction sites get lane
// work: each colour's sites are compacted into an LDS list with wave ballots.  Every staged
// value's (cos, sin) is evaluated once per tile, and an updated colour-0 site hands its new
// (cos, sin) straight to its colour-1 neighbours.  The sweep reads the source buffer and writes
// the tile's prediction sites into the destination buffer (sample values are equal in both).
//
// The field order ((left + right) + (up + down)), the site update, the Philox counters and the
// energy split by bond kind (colour-1 prediction sites: all four bonds; colour-0 prediction
// sites: bonds to colour-1 samples; sample-sample bonds: a constant of the data seeding the
// accumulator) are those of the compacted path, so the two paths agree bit for bit.
#pragma once

#include "mpr_sparse.hpp"

namespace mpr {

constexpr int kTileCols = 64;                     // plane columns per tile (128 grid columns)
// waves per block (one block per tile), a template parameter of the kernel: eight while the
// tiles fit the chip a few times over (a sweep is then bound by one block's latency, which
// more waves shorten: 3 % faster whole steps on 1024^2), four for more tiles (more blocks per
// CU overlap their phases: 21 % faster on 16384^2); two and sixteen were slower
constexpr int kTileWavesSmall = 8, kTileWavesLarge = 4;
constexpr int kTileWavesSwitch = 2048;             // tiles (of the base height) from which four waves are used

// base rows per tile: 16 when a staged element (raw value and its (cos, sin)) takes at most 12
// bytes or the functions are evaluated in double precision, else 8.  Four-wave blocks then take
// 28-67 KB of LDS; with double-precision functions their registers allow three waves per SIMD
// anyway, and 16-row tiles halve the staged halo (11 % faster kernels on 1024^2)
template <class S, class F> constexpr int tile_rows()
{
    return (sizeof(typename Store<S>::raw) + 2 * sizeof(F) <= 12 || sizeof(F) == 8) ? 16 : 8;
}
// Tile shapes: (waves per block, rows per tile).  The automatic rule takes eight-wave blocks on
// tiles of twice the base height (49-69 KB of LDS, two or three blocks per CU) when a grid fits
// the chip in about one round -- fewer and taller tiles stage and recompute less halo (10 %
// faster inference sweeps on 1024^2) -- and four-wave blocks on base-height tiles otherwise;
// the autotuner may pick the other two combinations (single-precision functions only: the
// tall tiles of double-precision values would exceed the LDS of a block).
enum { kShapeW4Base = 0, kShapeW8Tall = 1, kShapeW4Tall = 2, kShapeW8Base = 3, kTileShapes = 4 };
constexpr int shape_waves(int shape) { return (shape == kShapeW8Tall || shape == kShapeW8Base) ? 8 : 4; }
constexpr bool shape_tall(int shape) { return shape == kShapeW8Tall || shape == kShapeW4Tall; }
template <class S, class F, bool TALL> constexpr int tile_rows_for()
{
    return TALL ? 2 * tile_rows<S, F>() : tile_rows<S, F>();
}

struct TiledArgs {
    const int4* tiles;         // per tile (batched contexts): (gc, y0, k0, 1 if first of its gc)
    const GcDesc* gcs;
    const GcCtl* ctl;
    const RunCtl* run;
    const void* src;
    void* dst;
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
    double inv_piq;            // 1 / (pi q), as the other sweep kernels evaluate it
    int32_t n_gc, n_tiles, sweep_off;
    uint32_t key0, key1;
    int32_t single;            // one (grid, chain): tile b sits at row block b / ntx, column block b % ntx
    int32_t ntx;
    GcDesc g0;                 // one (grid, chain): its record, so no table read precedes the
                               // loads (geometry only: a reload with the same shapes keeps
                               // captured launches, so mask-dependent fields come from gcs)
};

template <class F> struct alignas(2 * sizeof(F)) CosSin { F c, s; };

template <class S, class F, int FLAGS, bool PER, int NW, bool TALL>
__global__ __launch_bounds__(NW * kWave) void k_tiled(TiledArgs a)
{
    using St = Store<S>;
    using M = Math<F>;
    using Raw = typename St::raw;
    using CS = CosSin<F>;
    constexpr int TY = tile_rows_for<S, F, TALL>(), TX = kTileCols;
    constexpr int R1 = TY + 4, W1 = TX + 4;       // colour-1 stage: rows y0-2 ..., columns k0-2 ...
    constexpr int R0 = TY + 2, W0 = TX + 2;       // colour-0 stage: rows y0-1 ..., columns k0-1 ...
    constexpr int N1 = R1 * W1, N0 = R0 * W0;
    constexpr int NT = kWave * NW;
    // a stage is read in passes of one 64-column row segment per wave (rows wave, wave + NW, ...)
    // plus one pass over the columns past the first 64 (4 for colour 1, 2 for colour 0)
    constexpr int I1 = (R1 + NW - 1) / NW, I0 = (R0 + NW - 1) / NW;
    constexpr int X1 = W1 - kWave, X0 = W0 - kWave;
    static_assert(X1 * R1 <= NT && X0 * R0 <= NT, "one pass covers the extra columns");
    // each wave compacts its prediction sites into its own list segment
    constexpr int SEG1 = (I1 + 1) * kWave, SEG0 = (I0 + 1) * kWave;
    constexpr uint32_t kRaw = (uint32_t)sizeof(Raw);
    constexpr bool FUSED = (FLAGS & F_ENERGY) != 0;   // this path sums energies in double precision
    // staged elements outside the grid: flagged as samples (never updated) with (cos, sin) = 0
    constexpr Raw kAbsent = (Raw)((Raw)1 << (8 * sizeof(Raw) - 1));

    __shared__ Raw raw1[N1];
    __shared__ CS cs1[N1];
    __shared__ Raw raw0[N0];
    __shared__ CS cs0[N0];
    __shared__ uint16_t list1[NW * SEG1], list0[NW * SEG0];
    __shared__ int count[2][NW];
    __shared__ double ctl_sh[2];
    __shared__ int64_t red[NW][3];

    if (blockDim.x != NT) return;                    // launched for another variant: no work
    const int tid = (int)threadIdx.x, lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lblock = xcd_block((int)blockIdx.x, (int)gridDim.x);
    int gc, y0, k0;
    bool first;
    if (a.single) {
        gc = 0;
        const int ty = lblock / a.ntx;
        y0 = ty * TY;
        k0 = (lblock - ty * a.ntx) * TX;
        first = lblock == 0;
    } else {
        const int4 t = a.tiles[lblock];
        gc = __builtin_amdgcn_readfirstlane(t.x);
        y0 = __builtin_amdgcn_readfirstlane(t.y);
        k0 = __builtin_amdgcn_readfirstlane(t.z);
        first = __builtin_amdgcn_readfirstlane(t.w) != 0;
    }

    GcDesc g;
    if (a.single) g = a.g0;
    else g = a.gcs[gc];
    const int H = g.H, W = g.W, pitch = g.pitch, wc = g.wc;
    const int ny = min(TY, H - y0), nk = min(TX, wc - k0);   // the tile proper, clipped to the grid
    const int plane_sz = H * pitch;
    const Rsrc rs = make_rsrc((const Raw*)a.src + g.plane_off, 2u * (uint32_t)plane_sz * kRaw);
    const Rsrc rd = make_rsrc((Raw*)a.dst + g.plane_off, 2u * (uint32_t)plane_sz * kRaw);

    // Stage elements.  Main passes: row r = wave + NW i (wave-uniform), column cc = lane; one
    // pass over the columns past the first 64: element tid of that strip.  The stage of colour
    // c with origin (y0 - h, k0 - h) covers rows r <= ny + 2h - 1 and columns cc <= nk + 2h - 1;
    // one wrap suffices for periodic grids (rows -2 .. H + 1, columns -2 .. wc + 1, H, wc >= 2).
    // Column part (per lane, once): plane column, and whether it is a grid site in a row of
    // parity 0 / 1; row part (per pass): grid row, whether it is in the grid, its parity.
    auto col_info = [&](int h, int cc, int& kk, bool& ev, bool& od) {
        kk = k0 - h + cc;
        const bool reg = cc <= nk + 2 * h - 1;
        if (PER) {
            kk = kk < 0 ? kk + wc : (kk >= wc ? kk - wc : kk);
            ev = od = reg;
        } else {
            ev = reg & (kk >= 0) & (2 * kk < W);
            od = reg & (kk >= 0) & (2 * kk + 1 < W);
        }
    };
    auto row_info = [&](int c, int h, int r, int& yy, bool& rok, int& par) {
        yy = y0 - h + r;
        rok = r <= ny + 2 * h - 1;
        if (PER) yy = yy < 0 ? yy + H : (yy >= H ? yy - H : yy);
        else rok &= (yy >= 0) & (yy < H);
        par = (yy + c) & 1;
    };

    // control state of this sweep (during an inference the previous sweep's control step,
    // applied here): wave 0 evaluates it for the block (the first tile's wave 0 also stores it)
    // and hands T and alpha over through LDS; its loads go out first, its arithmetic overlaps
    // the stage loads
    const int64_t s_abs = a.run->base_sweep + a.sweep_off;
    const uint32_t sweep = (uint32_t)s_abs;
    int acc_slot = 0;
    CtlFetch cf;
    if (wave == 0)
        cf = sweep_control_fetch(FUSED, true, gc, lane, a.ctl, a.run, a.ictl, a.gacc, a.n_gc, s_abs, acc_slot);

    // issue every stage load before anything waits on one
    int kk1, kx1, kk0, kx0;
    bool ev1, od1, evx1, odx1, ev0, od0, evx0, odx0;
    col_info(2, lane, kk1, ev1, od1);
    col_info(1, lane, kk0, ev0, od0);
    const int rx1 = tid / X1, cx1 = kWave + (tid - rx1 * X1);    // extra-column elements
    const int rx0 = tid / X0, cx0 = kWave + (tid - rx0 * X0);
    col_info(2, cx1, kx1, evx1, odx1);
    col_info(1, cx0, kx0, evx0, odx0);
    Raw v1[I1 + 1], v0[I0 + 1];
    bool ok1[I1 + 1], ok0[I0 + 1];
#pragma unroll
    for (int i = 0; i <= I1; ++i) {
        const bool main = i < I1;
        const int r = main ? wave + NW * i : rx1;
        int yy, par;
        bool rok;
        row_info(1, 2, r, yy, rok, par);
        const bool in = main ? r < R1 : tid < X1 * R1;
        ok1[i] = in & rok & (par ? (main ? od1 : odx1) : (main ? ev1 : evx1));
        const int kk = main ? kk1 : kx1;
        v1[i] = buf_load_one<St>(rs, ok1[i] ? (uint32_t)(plane_sz + yy * pitch + kk) * kRaw : kBufOOB);
    }
#pragma unroll
    for (int i = 0; i <= I0; ++i) {
        const bool main = i < I0;
        const int r = main ? wave + NW * i : rx0;
        int yy, par;
        bool rok;
        row_info(0, 1, r, yy, rok, par);
        const bool in = main ? r < R0 : tid < X0 * R0;
        ok0[i] = in & rok & (par ? (main ? od0 : odx0) : (main ? ev0 : evx0));
        const int kk = main ? kk0 : kx0;
        v0[i] = buf_load_one<St>(rs, ok0[i] ? (uint32_t)(yy * pitch + kk) * kRaw : kBufOOB);
    }

    if (wave == 0) {
        const GcCtl ctl = sweep_control_finish(cf, gc, a.gcs[gc], first, lane, a.run, a.ictl, a.gacc, a.econst,
                                               a.trace, a.n_gc, s_abs, a.J, a.acc_target, a.T_min,
                                               a.T_max);
        // the Boltzmann factor's scale as in the other sweep kernels: float path 2^(dE (-log2 e / T)),
        // double path exp(dE (-1 / T)); every wave reads it after the barrier
        if (lane == 0) { ctl_sh[0] = (sizeof(F) == 4) ? -1.4426950408889634 / ctl.T : -1.0 / ctl.T; ctl_sh[1] = ctl.alpha; }
    }
    const F q = (F)a.q;
    const F inv_piq = (F)a.inv_piq;

    // stage: raw values and (cos, sin); each wave compacts its prediction sites (ballots and a
    // running count) into its list segments
    int n_mine1 = 0, n_mine0 = 0;
    const bool lc1 = (lane >= 2) & (lane <= nk + 1), lcx1 = cx1 <= nk + 1;   // colour-1 list columns
#pragma unroll
    for (int i = 0; i <= I1; ++i) {
        const bool main = i < I1;
        const int r = main ? wave + NW * i : rx1;
        const bool in = main ? r < R1 : tid < X1 * R1;
        if (main && !in) continue;                       // wave-uniform
        const int e = r * W1 + (main ? lane : cx1);
        const Raw v = ok1[i] ? v1[i] : kAbsent;
        F s, c;
        M::sincos_rev(q * St::template value<F>(v), s, c);
        if (in) {
            raw1[e] = v;
            cs1[e] = CS{ok1[i] ? c : (F)0, ok1[i] ? s : (F)0};
        }
        const bool upd = ok1[i] & !St::sample(v) & (r >= 2) & (r <= ny + 1) & (main ? lc1 : lcx1);
        const uint64_t m = __ballot(upd);
        const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (upd) list1[wave * SEG1 + n_mine1 + below] = (uint16_t)e;
        n_mine1 += __popcll(m);
    }
#pragma unroll
    for (int i = 0; i <= I0; ++i) {
        const bool main = i < I0;
        const int r = main ? wave + NW * i : rx0;
        const bool in = main ? r < R0 : tid < X0 * R0;
        if (main && !in) continue;                       // wave-uniform
        const int e = r * W0 + (main ? lane : cx0);
        const Raw v = ok0[i] ? v0[i] : kAbsent;
        F s, c;
        M::sincos_rev(q * St::template value<F>(v), s, c);
        if (in) {
            raw0[e] = v;
            cs0[e] = CS{ok0[i] ? c : (F)0, ok0[i] ? s : (F)0};
        }
        const bool upd = ok0[i] & !St::sample(v);
        const uint64_t m = __ballot(upd);
        const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (upd) list0[wave * SEG0 + n_mine0 + below] = (uint16_t)e;
        n_mine0 += __popcll(m);
    }
    if (lane == 0) { count[0][wave] = n_mine0; count[1][wave] = n_mine1; }
    __syncthreads();

    const F J = (F)a.J;
    const F kexp = (F)ctl_sh[0];
    const F alpha = (F)ctl_sh[1];
    // list position i -> (wave segment, entry), from the prefix sums of the segment lengths
    int pre[2][NW + 1];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        pre[c][0] = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) pre[c][w + 1] = pre[c][w] + count[c][w];
    }
    auto entry = [&](const uint16_t* list, int seg, int c, int i) -> int {
        int w = 0, base = 0;
#pragma unroll
        for (int k = 1; k < NW; ++k)
            if (i >= pre[c][k]) { w = k; base = pre[c][k]; }
        return list[w * seg + (i - base)];
    };
    const int n0 = pre[0][NW], n1 = pre[1][NW];

    int n_acc = 0;
    int64_t e_hi = 0, e_lo = 0;
    const Rsrc ra = kAcc32<S> ? make_rsrc(a.acc32 + g.site_off, (uint32_t)(H * W) * 4u)
                              : make_rsrc(a.acc + g.site_off, (uint32_t)(H * W) * 8u);
    auto accumulate = [&](int c, int yy, int kk, Raw nv) {
        const uint32_t rank = (uint32_t)acc_rank(a.rk_mask, a.rk_base, g.rk_off, pitch, c, yy, kk);
        if constexpr (kAcc32<S>) {
            const uint32_t ao = rank * 4u;
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_amdgcn_raw_buffer_load_b32(ra, (int)ao, 0, 0) + acc_units<S>(nv),
                                                  ra, (int)ao, 0, 0);
        } else {
            const uint32_t ao = rank * 8u;
            buf_store_f64(ra, ao, buf_load_f64(ra, ao) + St::template value<double>(nv));
        }
    };

    // colour 0: the tile and its ring, from the old colour-1 stage
    for (int i = tid; i < n0; i += NT) {
        const int e = entry(list0, SEG0, 0, i);
        const int r = e / W0, cc = e - r * W0;
        int yy = y0 - 1 + r, kk = k0 - 1 + cc;
        if (PER) {
            yy = yy < 0 ? yy + H : (yy >= H ? yy - H : yy);
            kk = kk < 0 ? kk + wc : (kk >= wc ? kk - wc : kk);
        }
        const int p = yy & 1;
        const int b1 = (r + 1) * W1 + cc + 1;                 // same site in colour-1 stage coordinates
        const int il = b1 + p - 1, ir = b1 + p, iu = b1 - W1, id = b1 + W1;
        const CS nl = cs1[il], nr = cs1[ir], nu = cs1[iu], nd = cs1[id];
        const F Cf = (nl.c + nr.c) + (nu.c + nd.c);
        const F Sf = (nl.s + nr.s) + (nu.s + nd.s);
        const Raw v = raw0[e];
        const U4 rn = philox10(U4{(uint32_t)(yy * g.np + (kk >> 1)), sweep, (uint32_t)g.chain_word, 0u},
                               a.key0, a.key1);
        const uint32_t wa = (kk & 1) ? rn.z : rn.x, wb = (kk & 1) ? rn.w : rn.y;
        const SiteOut<S, F> o = hybrid_update<S, F>(St::template value<F>(v), true, Cf, Sf, q, inv_piq, J,
                                                    kexp, alpha, wa, wb);
        cs0[e] = CS{o.c, o.s};
        const bool own = (r >= 1) & (r <= ny) & (cc >= 1) & (cc <= nk);
        if (own) {
            const Raw nv = St::template encode<F>(o.u);
            const uint32_t elem = (uint32_t)(yy * pitch + kk);
            buf_store_one<St>(rd, elem * kRaw, nv);
            n_acc += (o.dec >> 1) & 1;
            if (FLAGS & F_ENERGY) {        // bonds to colour-1 samples only
                const bool ml = St::sample(raw1[il]), mr = St::sample(raw1[ir]);
                const bool mu = St::sample(raw1[iu]), md = St::sample(raw1[id]);
                const F Cs = ((ml ? nl.c : (F)0) + (mr ? nr.c : (F)0)) + ((mu ? nu.c : (F)0) + (md ? nd.c : (F)0));
                const F Ss = ((ml ? nl.s : (F)0) + (mr ? nr.s : (F)0)) + ((mu ? nu.s : (F)0) + (md ? nd.s : (F)0));
                const Fix2 f = fixed64x2((double)M::fma(o.c, Cs, o.s * Ss));
                e_hi += f.hi;
                e_lo += f.lo;
            }
            if (FLAGS & F_ACC) accumulate(0, yy, kk, nv);
            if (FLAGS & F_DEC) a.dec[g.site_off + (int64_t)yy * W + 2 * kk + p] = (uint8_t)o.dec;
        }
    }
    __syncthreads();

    // colour 1: the tile, from the new colour-0 stage
    for (int i = tid; i < n1; i += NT) {
        const int e = entry(list1, SEG1, 1, i);
        const int r = e / W1, cc = e - r * W1;
        const int yy = y0 - 2 + r, kk = k0 - 2 + cc;          // inside the grid: no wrap
        const int p = (yy + 1) & 1;
        const int b0 = (r - 1) * W0 + cc - 1;                 // same site in colour-0 stage coordinates
        const CS nl = cs0[b0 + p - 1], nr = cs0[b0 + p], nu = cs0[b0 - W0], nd = cs0[b0 + W0];
        const F Cf = (nl.c + nr.c) + (nu.c + nd.c);
        const F Sf = (nl.s + nr.s) + (nu.s + nd.s);
        const Raw v = raw1[e];
        const U4 rn = philox10(U4{(uint32_t)(yy * g.np + (kk >> 1)), sweep, (uint32_t)g.chain_word, 1u},
                               a.key0, a.key1);
        const uint32_t wa = (kk & 1) ? rn.z : rn.x, wb = (kk & 1) ? rn.w : rn.y;
        const SiteOut<S, F> o = hybrid_update<S, F>(St::template value<F>(v), true, Cf, Sf, q, inv_piq, J,
                                                    kexp, alpha, wa, wb);
        const Raw nv = St::template encode<F>(o.u);
        const uint32_t elem = (uint32_t)(plane_sz + yy * pitch + kk);
        buf_store_one<St>(rd, elem * kRaw, nv);
        n_acc += (o.dec >> 1) & 1;
        if (FLAGS & F_ENERGY) {
            const Fix2 f = fixed64x2((double)M::fma(o.c, Cf, o.s * Sf));
            e_hi += f.hi;
            e_lo += f.lo;
        }
        if (FLAGS & F_ACC) accumulate(1, yy, kk, nv);
        if (FLAGS & F_DEC) a.dec[g.site_off + (int64_t)yy * W + 2 * kk + p] = (uint8_t)o.dec;
    }

    if (FUSED) {
        n_acc = wave_sum_i32(n_acc);
        e_hi = wave_sum_i64(e_hi);
        e_lo = wave_sum_i64(e_lo);
        if (lane == 0) { red[wave][0] = e_hi; red[wave][1] = e_lo; red[wave][2] = (int64_t)n_acc; }
        __syncthreads();
        if (tid == 0) {             // wave 0 holds the accumulator slot of this sweep
            int64_t t0 = 0, t1 = 0, t2 = 0;
            for (int w = 0; w < NW; ++w) { t0 += red[w][0]; t1 += red[w][1]; t2 += red[w][2]; }
            unsigned long long* A = (unsigned long long*)(a.gacc + ((int64_t)acc_slot * a.n_gc + gc) * kAccPerGc) +
                                    (blockIdx.x & (kAccCopies - 1)) * kAccStride;
            atomicAdd(A, (unsigned long long)t0);
            atomicAdd(A + kAccWord, (unsigned long long)t1);
            atomicAdd(A + 2 * kAccWord, (unsigned long long)t2);
        }
    }
}

}  // namespace mpr
