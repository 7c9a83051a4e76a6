// mpr_device.hpp -- device code of the MPR library for gfx950: counter-based RNG, precision
// traits, the per-site hybrid update and the fused checkerboard sweep kernel.
//
// Layout.  A grid H x W is split by colour c = (x + y) & 1 into two planes of H rows; site
// (y, x) sits in plane c at row y, column k = x >> 1.  Neighbours of a colour-c site (y, k) are
// the other plane's (y, k + o - 1), (y, k + o), (y - 1, k), (y + 1, k) with o = (y + c) & 1, so a
// half-sweep is a 4-point stencil on the other plane.  Angles are stored in revolutions
// u = phi / 2 pi in [0, 1]; the sign bit marks a sample site (its value never changes), so no
// mask is read on the hot path.  A lane owns a pair of plane columns (2j, 2j + 1): one
// Philox4x32-10 call gives both sites of a pair their two uniforms.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mpr {

// ------------------------------------------------------------------ shared host/device types
struct GcDesc {            // one (grid, chain)
    int32_t H, W;          // grid sides
    int32_t wc;            // sites per plane row, rounded up: (W + 1) / 2
    int32_t np;            // lane pairs per plane row: (wc + 1) / 2
    int32_t pitch;         // elements per plane row (even, >= 2 np)
    int32_t chain_word;    // Philox counter word 2: grid * n_chains + chain
    int32_t grid;          // grid index
    int32_t item_begin;    // first work item of this (grid, chain)
    int32_t item_end;      // one past its last work item
    int32_t pad0;
    int64_t plane_off;     // element offset of its planes [2][H][pitch] in the state arrays
    int64_t site_off;      // offset into packed per-chain site arrays (row-major)
    int64_t grid_site_off; // offset into packed per-grid site arrays (z, mask, zhat)
    int64_t n_pred;        // prediction sites of the grid
    int64_t n_bonds;       // nearest-neighbour bonds of the grid
    double inv_n_pred;     // 1 / n_pred (0 without prediction sites), 1 / n_bonds: the control
    double inv_n_bonds;    // step multiplies instead of dividing (every wave evaluates it)
    int64_t rk_off;        // first entry of the grid's rank tables (see acc_rank)
};

struct Item {              // one wave's work: 60 output pairs x rows [y0, y1)
    int32_t gc, pair0, y0, y1;
    // the (grid, chain)'s plane geometry, repeated here so a wave can address its rows after a
    // single table read
    int64_t plane_off;
    int32_t H, W, np, pitch;
    // dy > 0: two half-wave items of at most kHalfOutPairs output pairs each, lanes 0-31 on rows
    // [y0, y1) and lanes 32-63 on rows [y0 + dy, y1 + dy) of the same columns (dy even); both
    // halves' rows with their halos, y0 - 2 ... y1 + dy + 1, lie inside the grid
    int32_t dy, pad;
};

struct GcCtl {             // per (grid, chain) control state, device resident
    double T, alpha;
    double T0, T_sum;
    double e_smp, e_sim, acc_rate;
    int64_t T_cnt;
};

struct RunCtl {            // per context, device resident
    int64_t base_sweep;    // Philox sweep index of sweep offset 0 of the next graph replay
    int64_t s_half;        // first sweep whose temperature enters the estimate
    int64_t trace_base;    // sweep index of trace entry 0 = first sweep of the inference
    int64_t trace_cap;     // trace entries per (grid, chain)
    int64_t n_infer;       // sweeps of the current inference: [trace_base, trace_base + n_infer)
    int64_t fixed;         // kFixT: the temperature stays (equilibration at a given T);
                           // kFixAlpha: the window stays too (measurement sweeps)
};
constexpr int kFixT = 1, kFixAlpha = 2;

// Inference sweeps in double-precision energy carry their own temperature control: sweep t of
// an inference adds its exact integer sums (energy words, accepted moves) into slot t % 3 of the
// per-(grid, chain) accumulators, and every wave of sweep t > 0 first applies the control step
// of sweep t - 1 from slot (t - 1) % 3 and the control state in slot (t - 1) & 1.  The first
// item of each (grid, chain) stores the new state in slot t & 1, the trace entry of sweep t - 1,
// and clears slot (t + 1) % 3 for the next sweep.  Kernel boundaries order all of it.  Atomics
// on one cache line serialise (about 12 ns each), so a slot holds kAccCopies copies and each of
// a copy's three words sits on a cache line of its own (a block adds its LDS-reduced sums to
// copy blockIdx % kAccCopies) and readers sum the copies (exact integers: the order does not
// matter).  One wave reads all copies, one per lane.
constexpr int kAccCopies = 64;
constexpr int kAccWord = 16;       // int64 words between the words of a copy (128 bytes)
constexpr int kAccStride = 3 * kAccWord;             // words 0, kAccWord, 2 kAccWord of a copy:
constexpr int kAccPerGc = kAccCopies * kAccStride;   // energy high, energy low, accepted moves

enum { F_ENERGY = 1, F_ACC = 2, F_DEC = 4 };
enum { DEC_OR = 1, DEC_ACCEPT = 2, DEC_OUTSIDE = 4 };

constexpr int kWave = 64;
constexpr int kPrefetchRows = 1;   // rows of both colours loaded ahead of use (2-4 measured no faster)
constexpr int kOutPairs = 60;      // output pairs per wave (2 halo lanes on each side)
constexpr int kHalfOutPairs = 28;  // output pairs per half wave of a two-half item
constexpr int kWavesPerBlock = 4;

struct SweepArgs {
    const Item* items;
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
    int64_t* e_part;           // per item: energy partial [2] (two-word fixed point, or float bits)
    int32_t* a_part;           // per item: accepted moves
    GcCtl* ictl;               // inference control states [2][n_gc]
    int64_t* gacc;             // inference accumulators [3][n_gc][kAccPerGc]
    double* trace;             // [n_gc][trace_cap][4]
    double acc_target, T_min, T_max;
    int32_t n_gc;
    int32_t n_items;
    int32_t sweep_off;         // sweep index = run->base_sweep + sweep_off
    uint32_t key0, key1;
    double q, J;
    int32_t periodic;
    int32_t pad;
};

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw, SC'11.  The key is uniform across a wave, so the key schedule
// stays in scalar registers; each round is two 32x32->64 multiplies and two 3-input xors.
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 n;
        // three-input xor in one v_bitop3_b32 (truth table 0x96)
        n.x = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96);
        n.y = (uint32_t)p1;
        n.z = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96);
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// ------------------------------------------------------------------ compute precision
// F = float: hardware transcendental instructions (v_sin_f32 / v_cos_f32 take revolutions,
// v_exp_f32 is 2^x), uniforms with 23 random bits.  F = double: ocml double functions.
template <class F> struct Math;

template <> struct Math<float> {
    static __device__ __forceinline__ void sincos_rev(float x, float& s, float& c)
    {
        s = __builtin_amdgcn_sinf(x);
        c = __builtin_amdgcn_cosf(x);
    }
    // exp(-dE / T) as 2^(dE * k) with k = -log2(e) / T
    static __device__ __forceinline__ float boltz(float dE, float k) { return __builtin_amdgcn_exp2f(dE * k); }
    static __device__ __forceinline__ float uniform(uint32_t w)
    {
        return __builtin_fmaf((float)(w >> 9), 1.0f / 8388608.0f, 1.0f / 16777216.0f);
    }
    // atan2(y, x) for y >= 0 (the local field's S is a sum of sines of angles in [0, pi]):
    // octant reduction to a = min/max in [0, 1] and the odd polynomial of Abramowitz & Stegun,
    // Handbook of Mathematical Functions, formula 4.4.49 (|error| <= 2e-8 on [0, 1]).
    // (0, 0) gives NaN; callers test for a vanishing field first.
    static __device__ __forceinline__ float atan2(float y, float x)
    {
        const float ax = __builtin_fabsf(x);
        const float mx = __builtin_fmaxf(ax, y), mn = __builtin_fminf(ax, y);
        const float t = mn * __builtin_amdgcn_rcpf(mx);
        const float t2 = t * t;
        float p = 0.0028662257f;
        p = __builtin_fmaf(p, t2, -0.0161657367f);
        p = __builtin_fmaf(p, t2, 0.0429096138f);
        p = __builtin_fmaf(p, t2, -0.0752896400f);
        p = __builtin_fmaf(p, t2, 0.1065626393f);
        p = __builtin_fmaf(p, t2, -0.1420889944f);
        p = __builtin_fmaf(p, t2, 0.1999355085f);
        p = __builtin_fmaf(p, t2, -0.3333314528f);
        float r = __builtin_fmaf(t * t2, p, t);
        r = (y > ax) ? 1.57079632679489662f - r : r;
        return (x < 0.0f) ? 3.14159265358979324f - r : r;
    }
    static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
};

template <> struct Math<double> {
    static __device__ __forceinline__ void sincos_rev(double x, double& s, double& c)
    {
        sincospi(2.0 * x, &s, &c);
    }
    static __device__ __forceinline__ double boltz(double dE, double k) { return exp(dE * k); }
    static __device__ __forceinline__ double uniform(uint32_t w)
    {
        return ((double)w + 0.5) * (1.0 / 4294967296.0);
    }
    static __device__ __forceinline__ double atan2(double y, double x) { return ::atan2(y, x); }
    static __device__ __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
};

// ------------------------------------------------------------------ storage precision
// Raw bit patterns; the sign bit is the sample flag.
template <class S> struct Store;

template <> struct Store<double> {
    using raw = uint64_t;
    struct pair { raw a, b; };
    static __device__ __forceinline__ pair load(const void* base, int idx)
    {
        const ulonglong2 v = *((const ulonglong2*)((const uint64_t*)base + idx));
        return {v.x, v.y};
    }
    static __device__ __forceinline__ void store(void* base, int idx, pair p)
    {
        *((ulonglong2*)((uint64_t*)base + idx)) = make_ulonglong2(p.a, p.b);
    }
    static __device__ __forceinline__ bool sample(raw r) { return (r >> 63) != 0; }
    template <class F> static __device__ __forceinline__ F value(raw r)
    {
        return (F)__longlong_as_double((long long)(r & 0x7fffffffffffffffull));
    }
    template <class F> static __device__ __forceinline__ raw encode(F u) { return (raw)__double_as_longlong((double)u); }
    // value rounded to storage precision, in compute precision
    template <class F> static __device__ __forceinline__ F round(F u) { return (F)(double)u; }
};

template <> struct Store<float> {
    using raw = uint32_t;
    struct pair { raw a, b; };
    static __device__ __forceinline__ pair load(const void* base, int idx)
    {
        const uint2 v = *((const uint2*)((const uint32_t*)base + idx));
        return {v.x, v.y};
    }
    static __device__ __forceinline__ void store(void* base, int idx, pair p)
    {
        *((uint2*)((uint32_t*)base + idx)) = make_uint2(p.a, p.b);
    }
    static __device__ __forceinline__ bool sample(raw r) { return (r >> 31) != 0; }
    template <class F> static __device__ __forceinline__ F value(raw r)
    {
        return (F)__uint_as_float(r & 0x7fffffffu);
    }
    template <class F> static __device__ __forceinline__ raw encode(F u) { return __float_as_uint((float)u); }
    template <class F> static __device__ __forceinline__ F round(F u) { return (F)(float)u; }
};

template <> struct Store<_Float16> {
    using raw = uint16_t;
    struct pair { raw a, b; };
    static __device__ __forceinline__ pair load(const void* base, int idx)
    {
        const uint32_t v = *((const uint32_t*)((const uint16_t*)base + idx));
        return {(raw)(v & 0xffffu), (raw)(v >> 16)};
    }
    static __device__ __forceinline__ void store(void* base, int idx, pair p)
    {
        *((uint32_t*)((uint16_t*)base + idx)) = (uint32_t)p.a | ((uint32_t)p.b << 16);
    }
    static __device__ __forceinline__ bool sample(raw r) { return (r >> 15) != 0; }
    template <class F> static __device__ __forceinline__ F value(raw r)
    {
        return (F)__builtin_bit_cast(_Float16, (uint16_t)(r & 0x7fffu));
    }
    template <class F> static __device__ __forceinline__ raw encode(F u)
    {
        return __builtin_bit_cast(uint16_t, (_Float16)(float)u);
    }
    template <class F> static __device__ __forceinline__ F round(F u) { return (F)(float)(_Float16)(float)u; }
};

// Averaging sweeps with FP16 storage sum into 32-bit words: every FP16 value in [0, 1] is a
// whole number of 2^-24 units (at most 2^24), so the words hold exact sums, which the host folds
// into the FP64 running sums after at most 128 sweeps (below 2^31).  Each partial sum of adding
// the values in double precision is a multiple of 2^-24 far below 2^29, exact as well: both
// give the same sums bit for bit, the words in half the bytes.  (16-bit fixed point,
// u = k / 32767, is not a dyadic fraction and keeps the FP64 sums.)
template <class S> constexpr bool kAcc32 = std::is_same_v<S, _Float16>;
template <class S> __device__ __forceinline__ uint32_t acc_units(typename Store<S>::raw r)
{
    return (uint32_t)(Store<S>::template value<float>(r) * 16777216.0f);
}

// 16-bit fixed point: 15 fraction bits with u = k / 32767 (uniform resolution 3.1e-5 of a turn,
// against FP16's 2^-11 just below 1) and the sample flag in bit 15.
struct Fix15 {};

template <> struct Store<Fix15> {
    using raw = uint16_t;
    struct pair { raw a, b; };
    static __device__ __forceinline__ pair load(const void* base, int idx)
    {
        const uint32_t v = *((const uint32_t*)((const uint16_t*)base + idx));
        return {(raw)(v & 0xffffu), (raw)(v >> 16)};
    }
    static __device__ __forceinline__ void store(void* base, int idx, pair p)
    {
        *((uint32_t*)((uint16_t*)base + idx)) = (uint32_t)p.a | ((uint32_t)p.b << 16);
    }
    static __device__ __forceinline__ bool sample(raw r) { return (r >> 15) != 0; }
    template <class F> static __device__ __forceinline__ F value(raw r)
    {
        return (F)(r & 0x7fffu) * (F)(1.0 / 32767.0);
    }
    template <class F> static __device__ __forceinline__ raw encode(F u)
    {
        const F k = __builtin_rint(u * (F)32767.0);
        return (raw)(k < (F)0 ? (F)0 : (k > (F)32767 ? (F)32767 : k));
    }
    template <class F> static __device__ __forceinline__ F round(F u) { return value<F>(encode<F>(u)); }
};

// ------------------------------------------------------------------ buffer addressing
// Plane accesses go through buffer resources: a byte offset at or past the resource's size reads
// zeros and drops writes, so lanes and rows outside the grid or the output range need no branch
// and every access issues, which lets the compiler wait for a load without also waiting for the
// stores issued after it.  A resource covers at most kBufMaxBytes (checked on the host).
using Rsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
constexpr uint32_t kBufMaxBytes = 0xFFFFFF00u;
constexpr uint32_t kBufOOB = 0xFFFFFF00u;          // offset that no resource covers

__device__ __forceinline__ Rsrc make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <class St>
__device__ __forceinline__ typename St::pair buf_load_pair(Rsrc r, uint32_t off)
{
    using raw = typename St::raw;
    if constexpr (sizeof(raw) == 8) {
        const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
        return {((uint64_t)v.y << 32) | v.x, ((uint64_t)v.w << 32) | v.z};
    } else if constexpr (sizeof(raw) == 4) {
        const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
        return {v.x, v.y};
    } else {
        const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
        return {(raw)(v & 0xffffu), (raw)(v >> 16)};
    }
}

template <class St>
__device__ __forceinline__ void buf_store_pair(Rsrc r, uint32_t off, typename St::pair p)
{
    using raw = typename St::raw;
    if constexpr (sizeof(raw) == 8) {
        u32x4_t v;
        v.x = (uint32_t)p.a; v.y = (uint32_t)(p.a >> 32); v.z = (uint32_t)p.b; v.w = (uint32_t)(p.b >> 32);
        __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, 0);
    } else if constexpr (sizeof(raw) == 4) {
        u32x2_t v;
        v.x = p.a; v.y = p.b;
        __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, 0, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32((uint32_t)p.a | ((uint32_t)p.b << 16), r, (int)off, 0, 0);
    }
}

__device__ __forceinline__ double2 buf_load_f64x2(Rsrc r, uint32_t off)
{
    const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    return make_double2(__longlong_as_double((long long)(((uint64_t)v.y << 32) | v.x)),
                        __longlong_as_double((long long)(((uint64_t)v.w << 32) | v.z)));
}

__device__ __forceinline__ double buf_load_f64(Rsrc r, uint32_t off)
{
    const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
    return __longlong_as_double((long long)(((uint64_t)v.y << 32) | v.x));
}

__device__ __forceinline__ void buf_store_f64(Rsrc r, uint32_t off, double d)
{
    const uint64_t b = (uint64_t)__double_as_longlong(d);
    u32x2_t v;
    v.x = (uint32_t)b; v.y = (uint32_t)(b >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, 0, 0);
}

__device__ __forceinline__ void buf_store_f64x2(Rsrc r, uint32_t off, double2 d)
{
    const uint64_t a = (uint64_t)__double_as_longlong(d.x), b = (uint64_t)__double_as_longlong(d.y);
    u32x4_t v;
    v.x = (uint32_t)a; v.y = (uint32_t)(a >> 32); v.z = (uint32_t)b; v.w = (uint32_t)(b >> 32);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, 0);
}

// ------------------------------------------------------------------ per-site hybrid update
// Input: current angle u (storage-rounded), local field (C, S) = sum_j (cos, sin)(2 pi q u_j),
// uniforms.  Output: new angle (storage-rounded), its (cos, sin)(2 pi q u), decision bits.
// Over-relaxation: the site energy is -J R cos(2 pi q u - psi), psi = atan2(S, C) in [0, pi]
// (all neighbour angles 2 pi q u_j lie in [0, pi], so S >= 0); the reflection
// u' = psi / (pi q) - u keeps it and is used when it stays in [0, 1].  Restricted Metropolis:
// proposal u + alpha (U_a - 1/2), rejected outside [0, 1], accepted iff
// U_b < exp(-(E(u_p) - E(u)) / T) with E(v) = -J (C cos 2 pi q v + S sin 2 pi q v) evaluated
// at the storage-rounded proposal.
template <class S, class F>
struct SiteOut {
    F u, c, s;
    int dec;
};

template <class S, class F>
__device__ __forceinline__ SiteOut<S, F> hybrid_update(F u, bool is_free, F C, F Sn, F q,
                                                      F inv_piq, F J, F kexp, F alpha,
                                                      uint32_t wa, uint32_t wb)
{
    using M = Math<F>;
    int dec = 0;
    // over-relaxation
    const bool has_field = (C != (F)0) | (Sn != (F)0);
    const F psi = M::atan2(Sn, C);
    const F ur = M::fma(psi, inv_piq, -u);
    const bool do_or = is_free & has_field & (ur >= (F)0) & (ur <= (F)1);
    F uc = do_or ? Store<S>::template round<F>(ur) : u;
    dec |= do_or ? DEC_OR : 0;
    F sc, cc;
    M::sincos_rev(q * uc, sc, cc);
    // restricted Metropolis
    const F up_raw = M::fma(alpha, M::uniform(wa) - (F)0.5, uc);
    const bool inside = is_free & (up_raw >= (F)0) & (up_raw <= (F)1);
    const F up = Store<S>::template round<F>(inside ? up_raw : uc);
    F sp, cp;
    M::sincos_rev(q * up, sp, cp);
    // dE = E(up) - E(uc) = J [C (cc - cp) + S (sc - sp)]
    const F dE = J * M::fma(C, cc - cp, Sn * (sc - sp));
    const bool acc = inside & (M::uniform(wb) < M::boltz(dE, kexp));
    dec |= inside ? (acc ? DEC_ACCEPT : 0) : (is_free ? DEC_OUTSIDE : 0);
    SiteOut<S, F> o;
    o.u = acc ? up : uc;
    o.c = acc ? cp : cc;
    o.s = acc ? sp : sc;
    o.dec = dec;
    return o;
}

// Two-word fixed-point image of an energy term, e ~ hi 2^-32 + lo 2^-64 (|e| < 2^18): both
// words are exact integers, so sums of them do not depend on the order of summation, and the
// quantum 2^-64 keeps e_sim + J (which can be ~1e-3 at low temperature) exact to the last bit
// of a double.  Rounding to integers uses the 1.5 * 2^52 shifter.
struct Fix2 { int64_t hi, lo; };

__device__ __forceinline__ int64_t round_to_i64(double t)    // |t| < 2^51
{
    const double s = t + 6755399441055744.0;
    return (int64_t)__double_as_longlong(s) - (int64_t)0x4338000000000000ll;
}

__device__ __forceinline__ Fix2 fixed64x2(double e)
{
    const double t = e * 4294967296.0;                        // exact
    const int64_t a = round_to_i64(t);
    const double r = (t - (double)a) * 4294967296.0;          // exact, |r| <= 2^31
    return Fix2{a, round_to_i64(r)};
}

// value of a two-word fixed-point sum hi 2^-32 + lo 2^-64 (hi split so every product is exact)
__host__ __device__ inline double fix2_value(int64_t hi, int64_t lo)
{
    const double k32 = 4294967296.0;
    const int64_t hi_top = hi >> 20, hi_bot = hi - (hi_top << 20);
    return (double)hi_top * 1048576.0 / k32 + ((double)hi_bot / k32 + (double)lo / (k32 * k32));
}

// Compact accumulators.  The FP64 running sums of the averaging sweeps are kept for prediction
// sites only: (grid, chain) gc's sums occupy acc[site_off + rank], rank = the site's position
// among its grid's prediction sites in the order (row y, colour c, plane column k).  Two tables
// per grid give the rank of any plane element: for each (y, c) row and each block of 64 plane
// columns, a bit mask of its prediction sites and the number of prediction sites before the block
// (tables entry rk_off + (2 y + c) nb + block, nb = pitch / 64).  The averaging sweeps then read
// and write 16 bytes per prediction site instead of per site.
__device__ __forceinline__ int64_t acc_rank(const uint64_t* rk_mask, const int32_t* rk_base,
                                            int64_t rk_off, int pitch, int c, int y, int k)
{
    const int64_t i = rk_off + (int64_t)(2 * y + c) * (pitch >> 6) + (k >> 6);
    const uint64_t below = (1ull << (k & 63)) - 1ull;
    return (int64_t)rk_base[i] + (int64_t)__popcll(rk_mask[i] & below);
}

// One step of the temperature and window control after an inference sweep (the multiplicative
// energy matching and the acceptance-driven window): e_sim from the exact bond-energy sum, T
// moved by the clamped ratio (e_smp + J) / (e_sim + J), alpha by A / A_target.  `c` holds the
// state used by the sweep and becomes the state of the next one; tr (if not null) receives the
// sweep's trace entry (e_sim, T, alpha, A).  `fixed` (kFixT, kFixAlpha bits) keeps T and / or
// alpha where they are.
__device__ inline void control_step(GcCtl& c, double e_sim, int64_t n_acc, const GcDesc& g,
                                    bool second_half, double J, double acc_target, double T_min,
                                    double T_max, double r_single, bool use_single, double* tr,
                                    int64_t fixed)
{
    const double A = g.n_pred > 0 ? (double)n_acc * g.inv_n_pred : acc_target;
    double r;
    if (use_single) r = r_single;
    else {
        const double num = c.e_smp + J, den = e_sim + J;
        r = den <= 1e-300 ? 2.0 : num / den;
    }
    if (tr) { tr[0] = e_sim; tr[1] = c.T; tr[2] = c.alpha; tr[3] = A; }
    if (second_half) { c.T_sum += c.T; c.T_cnt += 1; }
    r = fmin(fmax(r, 0.5), 2.0);
    if (!(fixed & kFixT)) c.T = fmin(fmax(c.T * r, T_min), T_max);
    if (!(fixed & kFixAlpha)) c.alpha = fmin(fmax(c.alpha * (A / acc_target), 1e-3), 1.0);
    c.e_sim = e_sim;
    c.acc_rate = A;
}

// ------------------------------------------------------------------ cross-lane shifts
// DPP wave shifts by one lane (a plain VALU move, no LDS crossbar): from_left(v) gives lane i
// the value of lane i-1, from_right(v) the value of lane i+1; lanes without a source get 0
// (bound_ctrl, so no move initialises the destination first).
__device__ __forceinline__ int dpp_from_left(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_from_right(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float from_left(float v) { return __int_as_float(dpp_from_left(__float_as_int(v))); }
__device__ __forceinline__ float from_right(float v) { return __int_as_float(dpp_from_right(__float_as_int(v))); }
__device__ __forceinline__ double from_left(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_from_left((int)(b & 0xffffffffll)), hi = dpp_from_left((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_right(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_from_right((int)(b & 0xffffffffll)), hi = dpp_from_right((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// XCD-aware block order: the dispatcher hands block b to XCD b % 8, each XCD with its own L2, so
// logical block numbers are dealt out in 8 contiguous runs, one per XCD.  Neighbouring work
// (adjacent row blocks, adjacent list entries) then shares one L2, and halo rows are fetched
// once per XCD instead of once per neighbour.  A bijection on [0, nb) for any nb.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int xcd = b % kXcds, local = b / kXcds;
    const int per = nb / kXcds, rem = nb % kXcds;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// Exact wave sum of a 32-bit integer whose total fits in 32 bits: DPP row shifts then row
// broadcasts (plain VALU moves, no LDS round trip); lane 63 ends with the total, returned
// wave-uniform.
__device__ __forceinline__ int wave_sum_i32(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15 -> rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31 -> rows 2, 3
    return __builtin_amdgcn_readlane(v, 63);
}

// Exact wave sum of a 64-bit integer of magnitude below 2^57 per lane: three 21-bit limbs
// (x = a 2^42 + b 2^21 + c, 0 <= b, c < 2^21), each limb's wave total fits in 32 bits.
__device__ __forceinline__ int64_t wave_sum_i64(int64_t x)
{
    const int c = (int)(x & 0x1FFFFF);
    const int b = (int)((x >> 21) & 0x1FFFFF);
    const int a = (int)(x >> 42);
    return ((int64_t)wave_sum_i32(a) << 42) + ((int64_t)wave_sum_i32(b) << 21) + (int64_t)wave_sum_i32(c);
}

// Control state used by a sweep of (grid, chain) gc.  Frozen (ctl) outside an inference or when
// the energy is summed in single precision; during an inference either applied here (apply:
// the control step of the previous sweep from its exact sums, by every wave alike; the lead
// wave stores the result, the trace entry, and resets the accumulator slot after next, whose
// copy 0 starts at econst[gc] if given) or read as stored by the kernel that applied it.
// Split in two so a kernel can issue the loads (fetch) long before it needs the result
// (finish); sweep_control does both.
struct CtlFetch {
    GcCtl c;               // the state to use, or to take the control step from
    int64_t eh, el, na;    // this lane's copy of the previous sweep's sums (apply only)
    int tm;                // sweep index within the inference
    bool apply;            // the previous sweep's control step is applied here
};

__device__ inline CtlFetch sweep_control_fetch(bool fused, bool apply, int gc, int lane,
                                               const GcCtl* ctl, const RunCtl* run,
                                               const GcCtl* ictl, const int64_t* gacc, int n_gc,
                                               int64_t s_abs, int& acc_slot)
{
    CtlFetch f;
    f.eh = f.el = f.na = 0;
    f.tm = 0;
    f.apply = false;
    acc_slot = 0;
    if (!fused) { f.c = ctl[gc]; return f; }
    const int64_t t = s_abs - run->trace_base;
    const bool infer = (t >= 0) & (t < run->n_infer);
    if (!infer) { f.c = ctl[gc]; return f; }
    const int tm = (int)t;
    f.tm = tm;
    acc_slot = tm % 3;
    if (!apply || tm == 0) { f.c = ictl[(tm & 1) * n_gc + gc]; return f; }
    f.apply = true;
    f.c = ictl[((tm - 1) & 1) * n_gc + gc];
    const int64_t* A = gacc + ((int64_t)((tm - 1) % 3) * n_gc + gc) * kAccPerGc;
    if (lane < kAccCopies) {
        f.eh = A[lane * kAccStride];
        f.el = A[lane * kAccStride + kAccWord];
        f.na = A[lane * kAccStride + 2 * kAccWord];
    }
    return f;
}

__device__ inline GcCtl sweep_control_finish(const CtlFetch& f, int gc, const GcDesc& g, bool lead,
                                             int lane, const RunCtl* run, GcCtl* ictl,
                                             int64_t* gacc, const int64_t* econst, double* trace,
                                             int n_gc, int64_t s_abs, double J, double acc_target,
                                             double T_min, double T_max)
{
    if (!f.apply) return f.c;
    const int tm = f.tm;
    GcCtl c = f.c;
    // 64 lanes: each 21-bit limb total stays below 2^27 for any int64 word
    const int64_t eh = wave_sum_i64(f.eh);
    const int64_t el = wave_sum_i64(f.el);
    const int64_t na = wave_sum_i64(f.na);
    double* tr = (lead && lane == 0) ? trace + ((int64_t)gc * run->trace_cap + (tm - 1)) * 4 : nullptr;
    control_step(c, -J * fix2_value(eh, el) * g.inv_n_bonds, na, g,
                 s_abs - 1 >= run->s_half, J, acc_target, T_min, T_max, 0.0, false, tr,
                 run->fixed);
    if (lead) {
        if (lane == 0) ictl[(tm & 1) * n_gc + gc] = c;
        if (lane < kAccCopies) {
            int64_t* z = gacc + ((int64_t)((tm + 1) % 3) * n_gc + gc) * kAccPerGc + lane * kAccStride;
            z[0] = (econst && lane == 0) ? econst[2 * gc] : 0;
            z[kAccWord] = (econst && lane == 0) ? econst[2 * gc + 1] : 0;
            z[2 * kAccWord] = 0;
        }
    }
    return c;
}

__device__ inline GcCtl sweep_control(bool fused, bool apply, int gc, const GcDesc& g, bool lead,
                                      int lane, const GcCtl* ctl, const RunCtl* run, GcCtl* ictl,
                                      int64_t* gacc, const int64_t* econst, double* trace,
                                      int n_gc, int64_t s_abs, double J, double acc_target,
                                      double T_min, double T_max, int& acc_slot)
{
    const CtlFetch f = sweep_control_fetch(fused, apply, gc, lane, ctl, run, ictl, gacc, n_gc, s_abs,
                                           acc_slot);
    return sweep_control_finish(f, gc, g, lead, lane, run, ictl, gacc, econst, trace, n_gc, s_abs, J,
                                acc_target, T_min, T_max);
}

// per-row data of one lane: (cos, sin) of both pair members, zero where the site is absent
template <class F> struct RowCS { F c0, s0, c1, s1; };

// ------------------------------------------------------------------ fused sweep kernel
// One wave = one work item: 64 lanes hold pairs pair0-2 .. pair0+61 of one (grid, chain);
// lanes 2..61 are output lanes.  The wave walks down rows y0-2 .. y1+1 keeping a 3-row window:
// the old colour-1 (cos, sin) feed the colour-0 update of the middle row, the new colour-0
// (cos, sin) of three rows feed the colour-1 update one row behind.  Halo lanes and rows
// repeat their neighbours' colour-0 updates bit for bit (same inputs, same counters), so
// items never exchange data within a sweep; the sweep reads `src` and writes `dst`.
// A two-half item (dy > 0) holds pairs pair0-2 .. pair0+29 in each half, output lanes 2..29 of
// the half, the upper half dy rows further down: the ragged last strips of two row blocks then
// fill one wave.  Rows k are the lower half's; the upper half's row k + dy enters only the
// lanes' address and counter offsets: every row of a two-half item lies inside the grid, so the
// row tests (and the periodic wrap) stay the same for both halves and wave-uniform.
// Single-precision functions: at least five waves per SIMD (at most 96 VGPRs; the compiler's own
// choice for some variants is four waves with up to 128), except the averaging variants, which
// hold an iteration's running sums in flight across its updates (four waves).
template <class S, class F, int FLAGS, bool ESINGLE, bool PER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((sizeof(F) == 4 && !(FLAGS & F_ACC)) ? 5 : 1))) void k_sweep(SweepArgs a)
{
    using St = Store<S>;
    using M = Math<F>;
    using Pair = typename St::pair;
    const int lane = threadIdx.x & (kWave - 1);
    const int lblock = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int wid = __builtin_amdgcn_readfirstlane(lblock * kWavesPerBlock + (int)(threadIdx.x >> 6));
    if (wid >= a.n_items) return;                 // whole waves leave together
    const Item it = a.items[wid];
    const GcDesc g = a.gcs[it.gc];
    const int64_t s_abs = a.run->base_sweep + a.sweep_off;
    const uint32_t sweep = (uint32_t)s_abs;

    // control state of this sweep: frozen, or (inference in double-precision energy) the
    // previous sweep's control step applied here from its exact sums
    constexpr bool FUSED = (FLAGS & F_ENERGY) && !ESINGLE;
    int acc_slot = 0;
    const GcCtl ctl = sweep_control(FUSED, true, it.gc, g, wid == g.item_begin, lane, a.ctl, a.run,
                                    a.ictl, a.gacc, nullptr, a.trace, a.n_gc, s_abs, a.J,
                                    a.acc_target, a.T_min, a.T_max, acc_slot);

    const F q = (F)a.q;
    const F J = (F)a.J;
    const F inv_piq = (F)(1.0 / (3.14159265358979323846 * a.q));
    const F alpha = (F)ctl.alpha;
    // Boltzmann factor exp(-dE/T): float path 2^(dE * (-log2 e / T)), double path exp(dE * (-1/T))
    const F kexp = (sizeof(F) == 4) ? (F)(-1.4426950408889634 / ctl.T) : (F)(-1.0 / ctl.T);

    const int H = it.H, np = it.np, pitch = it.pitch;
    const bool halves = it.dy > 0;
    const int hl = halves ? (lane & (kWave / 2 - 1)) : lane;      // lane within its half
    const int yoff = (halves & (lane >= kWave / 2)) ? it.dy : 0;  // this lane's row = k + yoff
    const int j = it.pair0 - 2 + hl;
    const bool in_range = (j >= 0) & (j < np);
    const int jj = PER ? ((j % np) + np) % np : j;        // periodic: W % 4 == 0, so wc is even
    const bool lane_ok = PER | in_range;
    const bool out_lane = (hl >= 2) & (hl < (halves ? kWave / 2 - 2 : kWave - 2)) & in_range;
    // site (y, c, m) of this lane has x = 4 jj + 2 m + ((y + c) & 1); it exists iff x < W
    const int wl = it.W - 4 * jj;
    const int col = 2 * jj;                              // plane column of member 0
    const int plane_sz = H * pitch;                      // 16 plane_sz <= kBufMaxBytes (host check)
    // lane offsets of row k: element (k + yoff) pitch + col of a plane, Philox counter word
    // (k + yoff) np + jj
    const int lane_elem = yoff * pitch + col;
    const int lane_ctr = yoff * np + jj;

    // this (grid, chain)'s two planes in the source and destination buffers, and its accumulators
    // (offsets count stored elements: the tag type of a fixed-point storage has no size of its own)
    using Raw = typename St::raw;
    constexpr uint32_t kRaw = (uint32_t)sizeof(Raw);
    const uint32_t gc_elems = 2u * (uint32_t)plane_sz;
    const Rsrc rs = make_rsrc((const Raw*)a.src + it.plane_off, gc_elems * kRaw);
    const Rsrc rd = make_rsrc((Raw*)a.dst + it.plane_off, gc_elems * kRaw);

    auto row_ok = [&](int y) -> bool { return PER | ((y >= 0) & (y < H)); };
    auto wrap = [&](int y) -> int { return PER ? (y < 0 ? y + H : (y >= H ? y - H : y)) : y; };
    // existence of member m at row parity p (= (y + c) & 1), rows aside: bit 2 m + p of ex_bits
    // (a value, not four addressable flags, so selecting one never goes through memory)
    const int ex_bits = lane_ok ? ((0 < wl) ? 1 : 0) | ((1 < wl) ? 2 : 0) | ((2 < wl) ? 4 : 0) | ((3 < wl) ? 8 : 0) : 0;
    // (par = (y + c) & 1 is passed by the caller: in the unrolled steady state it is a constant;
    // dy is even, so it is the parity of the upper half's row too)
    auto exists = [=](int y, int par, int m) -> bool {
        return (((ex_bits >> (2 * m + par)) & 1) != 0) & row_ok(y);
    };
    auto load_pair = [&](int c, int y) -> Pair {
        const uint32_t off = (lane_ok & row_ok(y)) ? (uint32_t)(c * plane_sz + wrap(y) * pitch + lane_elem) * kRaw : kBufOOB;
        return buf_load_pair<St>(rs, off);
    };
    auto cs_of = [&](Pair p, int y, int par) -> RowCS<F> {
        RowCS<F> r;
        F s, co;
        M::sincos_rev(q * St::template value<F>(p.a), s, co);
        const bool e0 = exists(y, par, 0), e1 = exists(y, par, 1);
        r.c0 = e0 ? co : (F)0;
        r.s0 = e0 ? s : (F)0;
        M::sincos_rev(q * St::template value<F>(p.b), s, co);
        r.c1 = e1 ? co : (F)0;
        r.s1 = e1 ? s : (F)0;
        return r;
    };

    // update both members of colour c at row y from the other colour's (cos, sin) rows up, mid,
    // dn; returns the new raw pair, the (cos, sin) of the new values (zero for absent sites),
    // the decisions, and the energy of this row's colour-c bonds with their final values
    auto update_row = [&](Pair old, const RowCS<F>& up, const RowCS<F>& mid, const RowCS<F>& dn,
                          int y, int c, int o, Pair& nw, RowCS<F>& ncs, int& da, int& db, F& e) {
        // horizontal neighbours (o = (y + c) & 1, the row parity): o == 0 -> member 0 uses (left
        // lane's member 1, own member 0), member 1 uses (own 0, own 1); o == 1 -> member 0 uses
        // (own 0, own 1), member 1 uses (own 1, right lane's member 0)
        F C0, S0, C1, S1;
        if (o == 0) {
            const F hc = from_left(mid.c1), hs = from_left(mid.s1);
            C0 = (hc + mid.c0) + (up.c0 + dn.c0);
            S0 = (hs + mid.s0) + (up.s0 + dn.s0);
            C1 = (mid.c0 + mid.c1) + (up.c1 + dn.c1);
            S1 = (mid.s0 + mid.s1) + (up.s1 + dn.s1);
        } else {
            const F hc = from_right(mid.c0), hs = from_right(mid.s0);
            C0 = (mid.c0 + mid.c1) + (up.c0 + dn.c0);
            S0 = (mid.s0 + mid.s1) + (up.s0 + dn.s0);
            C1 = (mid.c1 + hc) + (up.c1 + dn.c1);
            S1 = (mid.s1 + hs) + (up.s1 + dn.s1);
        }
        const bool ex0 = exists(y, o, 0), ex1 = exists(y, o, 1);
        const bool fr0 = ex0 & !St::sample(old.a);
        const bool fr1 = ex1 & !St::sample(old.b);
        // inference variants: the key words pass through an empty scalar-register asm, so the
        // compiler derives the round keys anew (scalar adds) at every call; hoisted out of the
        // row loop, the 20 round keys do not fit in scalar registers beside the energy sums'
        // state, and each call would reload them from VGPR lanes with VALU instructions (the
        // other variants keep them in scalar registers)
        uint32_t k0 = a.key0, k1 = a.key1;
        if constexpr ((FLAGS & F_ENERGY) != 0) __asm__ volatile("" : "+s"(k0), "+s"(k1));
        const U4 r = philox10(U4{(uint32_t)(wrap(y) * np + lane_ctr), sweep, (uint32_t)g.chain_word,
                                 (uint32_t)c},
                              k0, k1);
        const F u0 = St::template value<F>(old.a);
        const F u1 = St::template value<F>(old.b);
        const SiteOut<S, F> o0 = hybrid_update<S, F>(u0, fr0, C0, S0, q, inv_piq, J, kexp, alpha, r.x, r.y);
        const SiteOut<S, F> o1 = hybrid_update<S, F>(u1, fr1, C1, S1, q, inv_piq, J, kexp, alpha, r.z, r.w);
        nw.a = fr0 ? St::template encode<F>(o0.u) : old.a;
        nw.b = fr1 ? St::template encode<F>(o1.u) : old.b;
        ncs.c0 = ex0 ? o0.c : (F)0;
        ncs.s0 = ex0 ? o0.s : (F)0;
        ncs.c1 = ex1 ? o1.c : (F)0;
        ncs.s1 = ex1 ? o1.s : (F)0;
        da = o0.dec;
        db = o1.dec;
        e = M::fma(ncs.c0, C0, ncs.s0 * S0) + M::fma(ncs.c1, C1, ncs.s1 * S1);
    };

    int64_t e_hi = 0, e_lo = 0;   // two-word fixed-point energy sum (double-precision energy)
    float e_flt = 0.0f;           // single-precision energy sum
    int n_acc = 0;

    const int ya = it.y0, yb = it.y1;
    const RowCS<F> zero = {(F)0, (F)0, (F)0, (F)0};
    // loads run kPrefetchRows rows ahead of their use; rows past y1 + 1 are never used and not
    // loaded
    auto load_ahead = [&](int c, int y) -> Pair { return (y <= yb + 1) ? load_pair(c, y) : Pair{0, 0}; };

    // stores the new colour-c pair nv of row y (parity par = (y + c) & 1) with its decisions
    // da, db and accumulates the per-row outputs; keep (wave-uniform) says whether y is one of
    // the item's output rows.  The memory operations are issued either way (non-output lanes and
    // rows address past the resources, so their stores are dropped): every path through the
    // row loop then has the same count of stores behind the loads, and the compiler can wait for
    // the loads alone.
    auto finish = [&](int c, int y, int par, bool keep, const Pair& nv, int da, int db, F e)
        __attribute__((always_inline)) {
        const bool on = keep & out_lane;
        const uint32_t r = (uint32_t)(c * plane_sz + y * pitch + lane_elem);
        buf_store_pair<St>(rd, on ? r * kRaw : kBufOOB, nv);
        n_acc += on ? ((da >> 1) & 1) + ((db >> 1) & 1) : 0;
        if ((FLAGS & F_ENERGY) && c == 1) {
            const F eo = on ? e : (F)0;
            if (ESINGLE) e_flt += (float)eo;
            else { const Fix2 f = fixed64x2((double)eo); e_hi += f.hi; e_lo += f.lo; }
        }
        if ((FLAGS & F_DEC) && on) {
            uint8_t* d = a.dec + g.site_off + (int64_t)(y + yoff) * g.W + 4 * jj + par;
            if (exists(y, par, 0)) d[0] = (uint8_t)da;
            if (exists(y, par, 1)) d[2] = (uint8_t)db;
        }
    };

    // Averaging variant: the compact accumulators of the prediction sites of row y, colour c.
    // Which sites are prediction sites and their ranks do not depend on the update (the sample
    // flag of the old value is that of the new), so an iteration issues the loads of the running
    // sums of the two rows it stores before its updates (a scheduling barrier keeps them there),
    // and the updates' arithmetic hides them; the rank-table words those loads need are fetched
    // one iteration ahead.  Ranks: member 1 follows member 0 when both are prediction sites
    // (2 jj is even, so both share a mask block); lanes without output look up column 0 (halo
    // lanes' columns may lie outside the grid).  Measured: 100 averaging sweeps of the 256-grid
    // batch 177.6 -> 161.8 ms in FP32, 168.6 -> 140.4 ms in FP16.
    using AccSum = std::conditional_t<kAcc32<S>, uint32_t, double>;
    constexpr uint32_t kAccBytes = kAcc32<S> ? 4u : 8u;
    struct AccRow { uint32_t oa, ob; AccSum sa, sb; };
    struct RkRow { uint64_t m; int32_t b; };
    const Rsrc ra = kAcc32<S> ? make_rsrc(a.acc32 + g.site_off, (uint32_t)(it.H * it.W) * 4u)
                              : make_rsrc(a.acc + g.site_off, (uint32_t)(it.H * it.W) * 8u);
    const int ck = out_lane ? col : 0;
    const uint64_t below = (1ull << (ck & 63)) - 1ull;
    // rank-table words of row y (clamped into the grid: rows outside it are never stored)
    auto rk_fetch = [&](int c, int y) __attribute__((always_inline)) -> RkRow {
        const int yq = min(max(y + yoff, 0), H - 1);
        const int64_t i = g.rk_off + (int64_t)(2 * yq + c) * (pitch >> 6) + (ck >> 6);
        return RkRow{a.rk_mask[i], a.rk_base[i]};
    };
    auto acc_fetch = [&](int c, int y, int par, bool keep, const Pair& old, const RkRow& rk) __attribute__((always_inline)) -> AccRow {
        const bool on = keep & out_lane;
        const bool fa = on & exists(y, par, 0) & !St::sample(old.a);
        const bool fb = on & exists(y, par, 1) & !St::sample(old.b);
        const int64_t kr = (int64_t)rk.b + (int64_t)__popcll(rk.m & below);
        AccRow r;
        r.oa = fa ? (uint32_t)kr * kAccBytes : kBufOOB;
        r.ob = fb ? (uint32_t)(kr + fa) * kAccBytes : kBufOOB;
        if constexpr (kAcc32<S>) {
            r.sa = __builtin_amdgcn_raw_buffer_load_b32(ra, (int)r.oa, 0, 0);
            r.sb = __builtin_amdgcn_raw_buffer_load_b32(ra, (int)r.ob, 0, 0);
        } else {
            r.sa = buf_load_f64(ra, r.oa);
            r.sb = buf_load_f64(ra, r.ob);
        }
        return r;
    };
    auto acc_store = [&](const AccRow& r, const Pair& nv) __attribute__((always_inline)) {
        if constexpr (kAcc32<S>) {
            __builtin_amdgcn_raw_buffer_store_b32(r.sa + acc_units<S>(nv.a), ra, (int)r.oa, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(r.sb + acc_units<S>(nv.b), ra, (int)r.ob, 0, 0);
        } else {
            buf_store_f64(ra, r.oa, r.sa + St::template value<double>(nv.a));
            buf_store_f64(ra, r.ob, r.sb + St::template value<double>(nv.b));
        }
    };

    // Skewed pipeline: iteration k updates colour 0 at row k and colour 1 at row k - 2.  The two
    // updates share no data (colour 1 at row k - 2 needs the new colour 0 of rows k - 3 ... k - 1
    // only), so in the steady state they form one branch-free block the scheduler interleaves:
    // twice the independent work per wave of a one-row lag.  Both new rows are stored at the end
    // of their iteration (colour 1 first, measured 3 % faster than the other order), so no new
    // row is carried from one iteration to the next.
    // window: colour-1 old raw rows k-2 ... k+1 and (cos, sin) rows k-1 ... k+1; colour-0 new
    // (cos, sin) rows k-3 ... k
    Pair v0_cur, v0_next, r1_m2, r1_m1 = Pair{0, 0}, r1_0, r1_p1;
    RowCS<F> w1_m1, w1_0, w1_p1;
    RowCS<F> w0_m3, w0_m2 = zero, w0_m1 = zero, w0_0 = zero;
    RkRow rk1 = {0, 0}, rk0 = {0, 0};    // rank-table words of the rows the next iteration stores
    if constexpr ((FLAGS & F_ACC) != 0) {
        rk1 = rk_fetch(1, ya - 3);
        rk0 = rk_fetch(0, ya - 1);
    }

    r1_0 = load_pair(1, ya - 2);
    w1_0 = cs_of(r1_0, ya - 2, (ya - 1) & 1);
    r1_p1 = load_pair(1, ya - 1);
    w1_p1 = cs_of(r1_p1, ya - 1, ya & 1);
    v0_next = load_pair(0, ya - 1);
    Pair pf1[kPrefetchRows], pf0[kPrefetchRows];
#pragma unroll
    for (int d = 0; d < kPrefetchRows; ++d) {
        pf1[d] = load_ahead(1, ya + d);
        pf0[d] = load_ahead(0, ya + d);
    }

    // par = k & 1: colour 0 at row k and colour 1 at row k + 1 have parity par, colour 1 at
    // row k - 2 parity par ^ 1 (a constant in the unrolled steady state)
    auto step = [&](int k, int par, bool c0_rows_checked, bool do_c0, bool do_c1) __attribute__((always_inline)) {
        w1_m1 = w1_0; w1_0 = w1_p1;
        r1_m2 = r1_m1; r1_m1 = r1_0; r1_0 = r1_p1;
        w0_m3 = w0_m2; w0_m2 = w0_m1; w0_m1 = w0_0;
        v0_cur = v0_next;
        r1_p1 = pf1[0];
        v0_next = pf0[0];
#pragma unroll
        for (int d = 0; d + 1 < kPrefetchRows; ++d) {
            pf1[d] = pf1[d + 1];
            pf0[d] = pf0[d + 1];
        }
        pf1[kPrefetchRows - 1] = load_ahead(1, k + 1 + kPrefetchRows);
        pf0[kPrefetchRows - 1] = load_ahead(0, k + 1 + kPrefetchRows);
        const bool keep0 = do_c0 & (k >= ya) & (k < yb);
        AccRow q0, q1;
        if constexpr ((FLAGS & F_ACC) != 0) {
            q1 = acc_fetch(1, k - 2, par ^ 1, do_c1, r1_m2, rk1);
            q0 = acc_fetch(0, k, par, keep0, v0_cur, rk0);
            rk1 = rk_fetch(1, k - 1);
            rk0 = rk_fetch(0, k + 1);
            __builtin_amdgcn_sched_barrier(0);
        }
        Pair n0;
        int d0a, d0b;
        if (do_c0) w1_p1 = cs_of(r1_p1, k + 1, par);
        if (do_c0 && (!c0_rows_checked || row_ok(k))) {
            F e_unused;
            update_row(v0_cur, w1_m1, w1_0, w1_p1, k, 0, par, n0, w0_0, d0a, d0b, e_unused);
        } else {
            n0 = v0_cur;
            w0_0 = zero;
            d0a = d0b = 0;
        }
        Pair n1;
        int d1a, d1b;
        F e;
        if (do_c1) {
            RowCS<F> cs1;
            update_row(r1_m2, w0_m3, w0_m2, w0_m1, k - 2, 1, par ^ 1, n1, cs1, d1a, d1b, e);
        } else {
            n1 = Pair{0, 0};
            d1a = d1b = 0;
            e = (F)0;
        }
        finish(1, k - 2, par ^ 1, do_c1, n1, d1a, d1b, e);
        finish(0, k, par, keep0, n0, d0a, d0b, (F)0);
        if constexpr ((FLAGS & F_ACC) != 0) {
            acc_store(q1, n1);
            acc_store(q0, n0);
        }
    };
    // fill: colour 0 only (rows ya-1 ... ya+1); steady state: both colours, rows in the grid;
    // drain: colour 0 of row yb (if in the grid) and colour 1 of the last two rows
    int k = ya - 1;
    for (; k <= ya + 1 && k <= yb; ++k) step(k, k & 1, true, true, false);
    // steady state unrolled by two from an even row, so the row parities are constants (no
    // branch on them); unrolling by four renames the windows' registers too, but its 127 VGPRs
    // (four waves per SIMD instead of five) made the sweep 2-6 % slower
    if (k <= yb - 1 && (k & 1)) { step(k, 1, false, true, true); ++k; }
    for (; k + 1 <= yb - 1; k += 2) {
        step(k, 0, false, true, true);
        step(k + 1, 1, false, true, true);
    }
    for (; k <= yb - 1; ++k) step(k, k & 1, false, true, true);
    for (; k <= yb + 1; ++k) step(k, k & 1, true, k <= yb, k - 2 >= ya);

    // wave reductions (inference sweeps only): exact integer sums, or a fixed-order float tree
    if (!(FLAGS & F_ENERGY)) return;
    if (ESINGLE) {
        for (int off = kWave / 2; off > 0; off >>= 1) {
            n_acc += __shfl_xor(n_acc, off, kWave);
            e_flt += __shfl_xor(e_flt, off, kWave);
        }
    } else {
        n_acc = wave_sum_i32(n_acc);
        e_hi = wave_sum_i64(e_hi);
        e_lo = wave_sum_i64(e_lo);
    }
    if (FUSED) {
        unsigned long long* A = (unsigned long long*)(a.gacc + ((int64_t)acc_slot * a.n_gc + it.gc) * kAccPerGc);
        // a full block of one (grid, chain) adds once (block-uniform test: every wave of the
        // block takes the same branch, so all or none reach the barrier)
        const int b0 = lblock * kWavesPerBlock;
        const bool whole = (b0 + kWavesPerBlock <= a.n_items) &&
                           (a.items[b0].gc == a.items[b0 + kWavesPerBlock - 1].gc);
        if (whole) {
            __shared__ int64_t red[kWavesPerBlock][3];
            const int w = (int)(threadIdx.x >> 6);
            if (lane == 0) { red[w][0] = e_hi; red[w][1] = e_lo; red[w][2] = (int64_t)n_acc; }
            __syncthreads();
            if (threadIdx.x == 0) {
                int64_t s0 = 0, s1 = 0, s2 = 0;
                for (int k = 0; k < kWavesPerBlock; ++k) { s0 += red[k][0]; s1 += red[k][1]; s2 += red[k][2]; }
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
    } else if (lane == 0) {
        a.a_part[wid] = n_acc;
        if (FLAGS & F_ENERGY) {
            a.e_part[2 * wid] = ESINGLE ? (int64_t)__float_as_uint(e_flt) : e_hi;
            a.e_part[2 * wid + 1] = ESINGLE ? 0 : e_lo;
        }
    }
}

}  // namespace mpr
