// mpr.hip -- host runtime of the MPR library (C ABI declared in include/mpr.h) and the
// kernels around the sweep: validation and data map, sample energy, temperature / window
// control, averaging finalisation, checkpoint gather and scatter.
#include "mpr.h"
#include "mpr_device.hpp"
#include "mpr_sparse.hpp"
#include "mpr_tiled.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using namespace mpr;

namespace {

constexpr double kTwoPow32 = 4294967296.0;

// ------------------------------------------------------------------ load-time kernels
struct GridInfo {
    int64_t H, W;
    int64_t site_off;          // packed per-grid site offset
    uint64_t min_ord, max_ord; // order-preserving images of the sample min / max
    int64_t n_pred, n_sample;
    int64_t e_hi, e_lo;        // sample-bond energy, two-word fixed point (2^-32, 2^-64)
    int64_t n_sample_bonds;
    int32_t flags;             // 1: mask value > 1, 2: non-finite sample value
    int32_t pad;
    double zmin, zmax;
};

__device__ __forceinline__ uint64_t order_image(double d)
{
    const uint64_t b = (uint64_t)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
double order_inverse(uint64_t o)
{
    uint64_t b = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
    double d;
    std::memcpy(&d, &b, 8);
    return d;
}


template <class T> __device__ __forceinline__ T wave_sum(T v)
{
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// validation, sample min / max, site counts (one grid per blockIdx.y)
__global__ __launch_bounds__(256) void k_scan(GridInfo* gi, const double* z, const uint8_t* mask)
{
    GridInfo& G = gi[blockIdx.y];
    const int64_t n = G.H * G.W;
    uint64_t mn = ~0ull, mx = 0ull;
    int64_t n_pred = 0, n_samp = 0;
    int flags = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t m = mask[G.site_off + i];
        if (m > 1) flags |= 1;
        else if (m == 1) {
            const double v = z[G.site_off + i];
            if (!isfinite(v)) flags |= 2;
            else {
                const uint64_t o = order_image(v);
                mn = o < mn ? o : mn;
                mx = o > mx ? o : mx;
                ++n_samp;
            }
        } else ++n_pred;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const uint64_t a = __shfl_xor(mn, off, kWave), b = __shfl_xor(mx, off, kWave);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
        flags |= __shfl_xor(flags, off, kWave);
    }
    n_pred = wave_sum(n_pred);
    n_samp = wave_sum(n_samp);
    // combine the block's waves, then one set of atomics per block
    __shared__ uint64_t s_mn[4], s_mx[4];
    __shared__ int64_t s_np[4], s_ns[4];
    __shared__ int s_fl[4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & (kWave - 1)) == 0) { s_mn[w] = mn; s_mx[w] = mx; s_np[w] = n_pred; s_ns[w] = n_samp; s_fl[w] = flags; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            mn = s_mn[k] < mn ? s_mn[k] : mn;
            mx = s_mx[k] > mx ? s_mx[k] : mx;
            n_pred += s_np[k];
            n_samp += s_ns[k];
            flags |= s_fl[k];
        }
        atomicMin((unsigned long long*)&G.min_ord, (unsigned long long)mn);
        atomicMax((unsigned long long*)&G.max_ord, (unsigned long long)mx);
        atomicAdd((unsigned long long*)&G.n_pred, (unsigned long long)n_pred);
        atomicAdd((unsigned long long*)&G.n_sample, (unsigned long long)n_samp);
        if (flags) atomicOr(&G.flags, flags);
    }
}

// sample energy: sum over bonds with both ends sampled of cos[2 pi q (u_i - u_j)], FP64 terms,
// exact fixed-point accumulation (quantum 2^-32) so the result is independent of the launch
__global__ __launch_bounds__(256) void k_sample_energy(GridInfo* gi, const double* z,
                                                       const uint8_t* mask, double q, int periodic)
{
    GridInfo& G = gi[blockIdx.y];
    const int64_t H = G.H, W = G.W, n = H * W;
    const double lo = G.zmin, inv = 1.0 / (G.zmax - G.zmin);
    int64_t e_hi = 0, e_lo = 0, cnt = 0;
    // grid-stride loop with the site's (y, x) stepped along (one division per thread, not per
    // site)
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t dy = stride / W, dx = stride - dy * W;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t y = i / W, x = i - y * W;
    for (; i < n; i += stride, x += dx, y += dy) {
        if (x >= W) { x -= W; ++y; }
        if (mask[G.site_off + i] != 1) continue;
        const double ui = (z[G.site_off + i] - lo) * inv;
        int64_t nb[2];
        nb[0] = (x + 1 < W) ? i + 1 : (periodic ? y * W : -1);
        nb[1] = (y + 1 < H) ? i + W : (periodic ? x : -1);
        for (int k = 0; k < 2; ++k) {
            if (nb[k] < 0 || mask[G.site_off + nb[k]] != 1) continue;
            const double uj = (z[G.site_off + nb[k]] - lo) * inv;
            const Fix2 f = fixed64x2(cospi(2.0 * q * (ui - uj)));
            e_hi += f.hi;
            e_lo += f.lo;
            ++cnt;
        }
    }
    e_hi = wave_sum(e_hi);
    e_lo = wave_sum(e_lo);
    cnt = wave_sum(cnt);
    __shared__ int64_t s_h[4], s_l[4], s_c[4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & (kWave - 1)) == 0) { s_h[w] = e_hi; s_l[w] = e_lo; s_c[w] = cnt; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) { e_hi += s_h[k]; e_lo += s_l[k]; cnt += s_c[k]; }
        atomicAdd((unsigned long long*)&G.e_hi, (unsigned long long)e_hi);
        atomicAdd((unsigned long long*)&G.e_lo, (unsigned long long)e_lo);
        atomicAdd((unsigned long long*)&G.n_sample_bonds, (unsigned long long)cnt);
    }
}

// plane element -> raw stored value at load: samples get their mapped angle with the sign bit,
// prediction sites a uniform angle from the (tag 1, sweep 0) Philox counter
template <class S>
__global__ __launch_bounds__(256) void k_map_init(const GcDesc* gcs, const GridInfo* gi,
                                                  const double* z, const uint8_t* mask,
                                                  void* st0, void* st1,
                                                  uint32_t key0, uint32_t key1)
{
    using St = Store<S>;
    const GcDesc g = gcs[blockIdx.y];
    const GridInfo& G = gi[g.grid];
    const int64_t per_plane = (int64_t)g.H * g.pitch;
    const double lo = G.zmin, inv = 1.0 / (G.zmax - G.zmin);
    // element e = R pitch + k of the planes' 2 H rows (R = c H + y), stepped along the
    // grid-stride loop without a division per element
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t dR = stride / g.pitch, dk = stride - dR * g.pitch;
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t R = e / g.pitch, kk = e - R * g.pitch;
    for (; e < 2 * per_plane; e += stride, kk += dk, R += dR) {
        if (kk >= g.pitch) { kk -= g.pitch; ++R; }
        const int c = R >= g.H ? 1 : 0;
        const int y = (int)(R - (int64_t)c * g.H);
        const int k = (int)kk;
        const int x = 2 * k + ((y + c) & 1);
        typename St::raw v = 0;
        if (x < g.W) {
            const int64_t i = (int64_t)y * g.W + x;
            if (mask[g.grid_site_off + i]) {
                const double u = (z[g.grid_site_off + i] - lo) * inv;
                v = St::template encode<double>(u);
                v |= (typename St::raw)1 << (8 * sizeof(typename St::raw) - 1);
            } else {
                const U4 w = philox10(U4{(uint32_t)(y * g.np + (k >> 1)), 0u,
                                         (uint32_t)g.chain_word, (1u << 1) | (uint32_t)c},
                                      key0, key1);
                const uint32_t wa = (k & 1) ? w.z : w.x;
                v = St::template encode<double>(((double)wa + 0.5) * (1.0 / kTwoPow32));
            }
        }
        ((typename St::raw*)st0)[g.plane_off + e] = v;
        ((typename St::raw*)st1)[g.plane_off + e] = v;
    }
}

// Rank tables of the compact accumulators (acc_rank): for each grid, row y, colour c and block b
// of 64 plane columns, the bit mask of its prediction sites (mask value 0 inside the grid) and
// the number of prediction sites before the block in the order (y, c, k).  Built in four steps:
// masks and block counts; per (y, c) row an exclusive scan of its blocks' counts and the row's
// total; per grid an exclusive scan of the row totals; the row bases added to the blocks.
__global__ __launch_bounds__(256) void k_rank_count(const GcDesc* gcs, int n_chains, const uint8_t* mask,
                                                    uint64_t* rk_mask, int32_t* rk_base)
{
    const GcDesc g = gcs[blockIdx.y * n_chains];
    const int nb = g.pitch >> 6;
    const int64_t n = 2ll * g.H * nb;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int rowc = (int)(i / nb), b = (int)(i - (int64_t)rowc * nb);
        const int y = rowc >> 1, c = rowc & 1;
        const uint8_t* mrow = mask + g.grid_site_off + (int64_t)y * g.W;
        uint64_t m = 0;
        for (int t = 0; t < 64; ++t) {
            const int x = 2 * (64 * b + t) + ((y + c) & 1);
            if (x < g.W && mrow[x] == 0) m |= 1ull << t;
        }
        rk_mask[g.rk_off + i] = m;
        rk_base[g.rk_off + i] = __popcll(m);
    }
}

__global__ __launch_bounds__(256) void k_rank_rows(const GcDesc* gcs, int n_chains, int32_t* rk_base,
                                                   int32_t* row_tot, const int64_t* row_off)
{
    const GcDesc g = gcs[blockIdx.y * n_chains];
    const int nb = g.pitch >> 6;
    for (int rowc = blockIdx.x * blockDim.x + threadIdx.x; rowc < 2 * g.H; rowc += gridDim.x * blockDim.x) {
        int32_t* p = rk_base + g.rk_off + (int64_t)rowc * nb;
        int32_t run = 0;
        for (int b = 0; b < nb; ++b) { const int32_t v = p[b]; p[b] = run; run += v; }
        row_tot[row_off[blockIdx.y] + rowc] = run;
    }
}

// one block per grid: exclusive scan of the grid's 2 H row totals, in tiles of 1024
__global__ __launch_bounds__(256) void k_rank_rowscan(const GcDesc* gcs, int n_chains, int32_t* row_tot,
                                                      const int64_t* row_off)
{
    const GcDesc g = gcs[blockIdx.x * n_chains];
    int32_t* p = row_tot + row_off[blockIdx.x];
    const int n = 2 * g.H, tid = threadIdx.x;
    __shared__ int32_t sh[256];
    int32_t carry = 0;
    for (int base = 0; base < n; base += 1024) {
        int32_t v[4], t = 0;
        for (int j = 0; j < 4; ++j) {
            const int i = base + 4 * tid + j;
            v[j] = i < n ? p[i] : 0;
            t += v[j];
        }
        sh[tid] = t;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int32_t add = tid >= off ? sh[tid - off] : 0;
            __syncthreads();
            sh[tid] += add;
            __syncthreads();
        }
        int32_t r = sh[tid] - t + carry;
        const int32_t total = sh[255];
        __syncthreads();
        for (int j = 0; j < 4; ++j) {
            const int i = base + 4 * tid + j;
            if (i < n) p[i] = r;
            r += v[j];
        }
        carry += total;
    }
}

__global__ __launch_bounds__(256) void k_rank_add(const GcDesc* gcs, int n_chains, int32_t* rk_base,
                                                  const int32_t* row_tot, const int64_t* row_off)
{
    const GcDesc g = gcs[blockIdx.y * n_chains];
    const int nb = g.pitch >> 6;
    const int64_t n = 2ll * g.H * nb;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        rk_base[g.rk_off + i] += row_tot[row_off[blockIdx.y] + (int)(i / nb)];
}

__global__ __launch_bounds__(256) void k_copy_z(const GridInfo* gi, const double* z, double* zcopy)
{
    const GridInfo& G = gi[blockIdx.y];
    const int64_t n = G.H * G.W;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        zcopy[G.site_off + i] = z[G.site_off + i];
}

// ------------------------------------------------------------------ control kernels
__global__ void k_infer_begin(GcCtl* ctl, GcCtl* ictl, int64_t* gacc, const int64_t* econst,
                              int n_gc, double J, double T_min, double T_max, RunCtl* run,
                              int64_t s_half, int64_t trace_base, int64_t trace_cap, int64_t n_infer,
                              int fixed)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        run->s_half = s_half; run->trace_base = trace_base; run->trace_cap = trace_cap;
        run->n_infer = n_infer;
        run->fixed = fixed;
    }
    if (i < 3 * n_gc * kAccCopies) {                // thread i clears copy i of all slots
        int64_t* z = gacc + (int64_t)i * kAccStride;
        const int gc = (i / kAccCopies) % n_gc;
        const bool first = econst && (i % kAccCopies) == 0;   // copy 0 starts at the constant
        z[0] = first ? econst[2 * gc] : 0;
        z[kAccWord] = first ? econst[2 * gc + 1] : 0;
        z[2 * kAccWord] = 0;
    }
    if (i >= n_gc) return;
    GcCtl& c = ctl[i];
    // the matching starts from T_0 = clamp(4 (e_smp + J)); an equilibration keeps its T
    const double T0 = (fixed & kFixT) ? c.T : fmin(fmax(4.0 * (c.e_smp + J), T_min), T_max);
    c.T0 = T0;
    c.T = T0;
    c.T_sum = 0.0;
    c.T_cnt = 0;
    ictl[i] = c;                                   // state of inference sweep 0
}

// after n inference sweeps: with in-sweep control (double-precision energy) apply the control
// step of the last sweep and copy the state out; then T-hat = mean of the recorded temperatures
__global__ void k_infer_end(const GcDesc* gcs, GcCtl* ctl, const GcCtl* ictl, const int64_t* gacc,
                            double* trace, const RunCtl* run, int n_gc, int fused, int64_t n,
                            double J, double acc_target, double T_min, double T_max)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_gc) return;
    GcCtl c = ctl[i];
    if (fused && n > 0) {
        const int t = (int)(n - 1);
        c = ictl[(t & 1) * n_gc + i];
        const int64_t* A = gacc + ((int64_t)(t % 3) * n_gc + i) * kAccPerGc;
        int64_t eh = 0, el = 0, na = 0;
        for (int k = 0; k < kAccCopies; ++k) {
            eh += A[k * kAccStride];
            el += A[k * kAccStride + kAccWord];
            na += A[k * kAccStride + 2 * kAccWord];
        }
        const GcDesc g = gcs[i];
        control_step(c, -J * fix2_value(eh, el) * g.inv_n_bonds, na, g,
                     run->trace_base + t >= run->s_half, J, acc_target, T_min, T_max, 0.0, false,
                     trace + ((int64_t)i * run->trace_cap + t) * 4, run->fixed);
    }
    if (!(run->fixed & kFixT)) c.T = c.T_cnt > 0 ? c.T_sum / (double)c.T_cnt : c.T0;
    ctl[i] = c;
}

// temperature from a sampled energy-temperature curve of the unconditional model (T ascending):
// the T at which the curve reaches the (grid, chain)'s sample energy, linear between the first
// bracketing pair of points from the low end, clamped to the end points
__global__ void k_curve_temperature(GcCtl* ctl, int n_gc, const double* T, const double* e, int n_T)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_gc) return;
    const double et = ctl[i].e_smp;
    double r = T[n_T - 1];
    if (n_T < 2 || et <= e[0]) r = T[0];
    else
        for (int k = 0; k + 1 < n_T; ++k)
            if (et <= e[k + 1]) {
                const double de = e[k + 1] - e[k];
                r = de > 0.0 ? T[k] + (T[k + 1] - T[k]) * ((et - e[k]) / de) : T[k];
                break;
            }
    ctl[i].T = r;
}

// each (grid, chain)'s temperature into a plain array (the allocation-free curve entry point
// reads it back from its static scratch)
__global__ void k_gather_T(const GcCtl* ctl, int n_gc, double* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_gc) out[i] = ctl[i].T;
}

__global__ void k_advance(RunCtl* run, int64_t n) { run->base_sweep += n; }
__global__ void k_set_base(RunCtl* run, int64_t v) { run->base_sweep = v; }

// one block per (grid, chain): sum the per-item partials in item order, then move T and alpha
template <bool ESINGLE>
__global__ __launch_bounds__(1024) void k_control(const GcDesc* gcs, GcCtl* ctl, const RunCtl* run,
                                                  const int64_t* e_part, const int32_t* a_part,
                                                  double* trace, int32_t sweep_off, double J,
                                                  double acc_target, double T_min, double T_max)
{
    // one block per (grid, chain): strided sums of the item partials (four loads in flight per
    // thread), a butterfly inside each wave, the waves in order (exact for the integer words;
    // a fixed order for the single-precision sum)
    __shared__ int64_t s_e[16], s_l[16], s_a[16];
    __shared__ float s_f[16];
    const GcDesc g = gcs[blockIdx.x];
    const int nt = (int)blockDim.x;
    int64_t e = 0, el = 0, na = 0;
    float ef = 0.0f;
    int i = g.item_begin + (int)threadIdx.x;
    for (; i + 3 * nt < g.item_end; i += 4 * nt) {
        int64_t h[4], l[4];
        int32_t n[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            h[u] = e_part[2 * (i + u * nt)];
            l[u] = e_part[2 * (i + u * nt) + 1];
            n[u] = a_part[i + u * nt];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (ESINGLE) ef += __uint_as_float((uint32_t)h[u]);
            else { e += h[u]; el += l[u]; }
            na += n[u];
        }
    }
    for (; i < g.item_end; i += nt) {
        if (ESINGLE) ef += __uint_as_float((uint32_t)e_part[2 * i]);
        else { e += e_part[2 * i]; el += e_part[2 * i + 1]; }
        na += a_part[i];
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        if (ESINGLE) ef += __shfl_xor(ef, off, kWave);
        else { e += __shfl_xor(e, off, kWave); el += __shfl_xor(el, off, kWave); }
        na += __shfl_xor(na, off, kWave);
    }
    const int w = (int)threadIdx.x >> 6;
    if ((threadIdx.x & (kWave - 1)) == 0) { s_e[w] = e; s_l[w] = el; s_a[w] = na; s_f[w] = ef; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < nt / kWave; ++k) { e += s_e[k]; el += s_l[k]; na += s_a[k]; ef += s_f[k]; }
    }
    if (threadIdx.x != 0) return;
    GcCtl c = ctl[blockIdx.x];
    const int64_t s = run->base_sweep + sweep_off;
    double e_sim, r_single = 0.0;
    if (ESINGLE) {
        const float es = -(float)J * ef / (float)g.n_bonds;
        const float num = (float)c.e_smp + (float)J, den = es + (float)J;
        r_single = (double)(den <= 1e-30f ? 2.0f : num / den);
        e_sim = (double)es;
    } else {
        e_sim = -J * fix2_value(e, el) * g.inv_n_bonds;
    }
    const int64_t t = s - run->trace_base;
    double* tr = (t >= 0 && t < run->trace_cap) ? trace + ((int64_t)blockIdx.x * run->trace_cap + t) * 4 : nullptr;
    control_step(c, e_sim, na, g, s >= run->s_half, J, acc_target, T_min, T_max, r_single,
                 ESINGLE, tr, run->fixed);
    ctl[blockIdx.x] = c;
}

// ------------------------------------------------------------------ finalise / checkpoint
template <class S>
__global__ __launch_bounds__(256) void k_finalize(const GcDesc* gcs, const GridInfo* gi,
                                                  const void* st, const double* acc,
                                                  const uint64_t* rk_mask, const int32_t* rk_base,
                                                  const double* zcopy, double* zhat,
                                                  int n_chains, int64_t n_avg)
{
    using St = Store<S>;
    const int grid = blockIdx.y;
    const GridInfo& G = gi[grid];
    const GcDesc g0 = gcs[grid * n_chains];
    const int64_t n = G.H * G.W;
    const int64_t per_plane = (int64_t)g0.H * g0.pitch;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = i / G.W, x = i - y * G.W;
        const int c = (int)((x + y) & 1);
        const int64_t e = c * per_plane + y * g0.pitch + (x >> 1);
        const typename St::raw v = ((const typename St::raw*)st)[g0.plane_off + e];
        double out;
        if (St::sample(v)) out = zcopy[G.site_off + i];
        else {
            double m = 0.0;
            const int64_t rank = acc_rank(rk_mask, rk_base, g0.rk_off, g0.pitch, c, (int)y, (int)(x >> 1));
            for (int ch = 0; ch < n_chains; ++ch)
                m += acc[gcs[grid * n_chains + ch].site_off + rank] / (double)n_avg;
            m /= (double)n_chains;
            out = G.zmin + (G.zmax - G.zmin) * m;
        }
        zhat[G.site_off + i] = out;
    }
}

template <class S>
__global__ __launch_bounds__(256) void k_get_state(const GcDesc* gcs, const void* st,
                                                   const double* acc, const uint64_t* rk_mask,
                                                   const int32_t* rk_base, double* u_out,
                                                   double* acc_out)
{
    using St = Store<S>;
    const GcDesc g = gcs[blockIdx.y];
    const int64_t n = (int64_t)g.H * g.W;
    const int64_t per_plane = (int64_t)g.H * g.pitch;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = i / g.W, x = i - y * g.W;
        const int64_t e = g.plane_off + ((x + y) & 1) * per_plane + y * g.pitch + (x >> 1);
        const typename St::raw v = ((const typename St::raw*)st)[e];
        if (u_out) u_out[g.site_off + i] = St::template value<double>(v);
        if (acc_out)
            acc_out[g.site_off + i] = St::sample(v) ? 0.0
                : acc[g.site_off + acc_rank(rk_mask, rk_base, g.rk_off, g.pitch, (int)((x + y) & 1), (int)y, (int)(x >> 1))];
    }
}

// check (mode 0) or write (mode 1) prediction-site angles; flag 1 = value outside [0, 1]
template <class S>
__global__ __launch_bounds__(256) void k_set_state(const GcDesc* gcs, void* st, double* acc,
                                                   const uint64_t* rk_mask, const int32_t* rk_base,
                                                   const double* u_in, const double* acc_in,
                                                   int* flag, int mode)
{
    using St = Store<S>;
    const GcDesc g = gcs[blockIdx.y];
    const int64_t n = (int64_t)g.H * g.W;
    const int64_t per_plane = (int64_t)g.H * g.pitch;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = i / g.W, x = i - y * g.W;
        const int64_t e = g.plane_off + ((x + y) & 1) * per_plane + y * g.pitch + (x >> 1);
        typename St::raw* p = (typename St::raw*)st + e;
        if (St::sample(*p)) continue;
        if (u_in) {
            const double u = u_in[g.site_off + i];
            if (mode == 0) {
                if (!(u >= 0.0 && u <= 1.0)) atomicOr(flag, 1);
            } else {
                *p = St::template encode<double>(u);
            }
        }
        if (acc_in && mode == 1)
            acc[g.site_off + acc_rank(rk_mask, rk_base, g.rk_off, g.pitch, (int)((x + y) & 1), (int)y, (int)(x >> 1))] =
                acc_in[g.site_off + i];
    }
}

// ------------------------------------------------------------------ site lists (compacted path)
// Prediction sites of plane c, row y of grid gr (its first chain's planes: all chains share
// the mask): those with x = 2k + ((y + c) & 1) < W and no sample flag.
template <class S>
__device__ __forceinline__ bool listed_site(const typename Store<S>::raw* row, int k, int par, int W, int pitch)
{
    return (k < pitch) && (2 * k + par < W) && !Store<S>::sample(row[k < pitch ? k : 0]);
}

template <class T> __device__ __forceinline__ T block_sum256(T v, T* sh)
{
    v = wave_sum(v);
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    T t = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return t;
}

// row counts: block (row y, grid gr * 2 + colour c), 256 threads
template <class S>
__global__ __launch_bounds__(256) void k_list_count(const GcDesc* gcs, int n_chains, const void* st,
                                                    int32_t* row_cnt, const int64_t* row_off)
{
    using St = Store<S>;
    __shared__ int sh[4];
    const int gr = blockIdx.y >> 1, c = blockIdx.y & 1;
    const GcDesc g = gcs[gr * n_chains];
    const int y = blockIdx.x;
    if (y >= g.H) return;                                    // uniform over the block
    const typename St::raw* row = (const typename St::raw*)st + g.plane_off +
                                  ((int64_t)c * g.H + y) * g.pitch;
    int cnt = 0;
    for (int k0 = 0; k0 < g.pitch; k0 += 256)
        cnt += listed_site<S>(row, k0 + (int)threadIdx.x, (y + c) & 1, g.W, g.pitch) ? 1 : 0;
    cnt = block_sum256(cnt, sh);
    if (threadIdx.x == 0) row_cnt[row_off[gr] + (int64_t)c * g.H + y] = cnt;
}

// exclusive scan of the row counts of (grid, colour) = blockIdx.x into row starts (in place);
// totals[blockIdx.x] receives the number of listed sites
__global__ __launch_bounds__(256) void k_list_scan(const GcDesc* gcs, int n_chains, int32_t* row_cnt,
                                                   const int64_t* row_off, int32_t* totals)
{
    __shared__ int sh[4];
    const int gr = blockIdx.x >> 1, c = blockIdx.x & 1;
    const GcDesc g = gcs[gr * n_chains];
    int32_t* r = row_cnt + row_off[gr] + (int64_t)c * g.H;
    int base = 0;
    for (int y0 = 0; y0 < g.H; y0 += 256) {
        const int y = y0 + (int)threadIdx.x;
        const int v = y < g.H ? r[y] : 0;
        // inclusive scan inside the wave, then across the four waves
        int inc = v;
        const int lane = threadIdx.x & (kWave - 1);
        for (int off = 1; off < kWave; off <<= 1) {
            const int t = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += t;
        }
        if (lane == kWave - 1) sh[threadIdx.x >> 6] = inc;
        __syncthreads();
        int wbase = 0;
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wbase += sh[w];
        const int total = sh[0] + sh[1] + sh[2] + sh[3];
        if (y < g.H) r[y] = base + wbase + inc - v;
        base += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = base;
}

// fill: block (row y, grid * 2 + colour) writes its row's sites in column order at
// list_base[grid * 2 + colour] + row start
template <class S>
__global__ __launch_bounds__(256) void k_list_fill(const GcDesc* gcs, int n_chains, const void* st,
                                                   const int32_t* row_start, const int64_t* row_off,
                                                   const int64_t* list_base, uint32_t* sites)
{
    using St = Store<S>;
    __shared__ int sh[4];
    const int gr = blockIdx.y >> 1, c = blockIdx.y & 1;
    const GcDesc g = gcs[gr * n_chains];
    const int y = blockIdx.x;
    if (y >= g.H) return;                                    // uniform over the block
    const typename St::raw* row = (const typename St::raw*)st + g.plane_off +
                                  ((int64_t)c * g.H + y) * g.pitch;
    int64_t pos = list_base[blockIdx.y] + row_start[row_off[gr] + (int64_t)c * g.H + y];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
    for (int k0 = 0; k0 < g.pitch; k0 += 256) {
        const int k = k0 + (int)threadIdx.x;
        const bool f = listed_site<S>(row, k, (y + c) & 1, g.W, g.pitch);
        const unsigned long long m = __ballot(f);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) sh[w] = __popcll(m);
        __syncthreads();
        int wbase = 0;
        for (int i = 0; i < w; ++i) wbase += sh[i];
        const int total = sh[0] + sh[1] + sh[2] + sh[3];
        if (f) sites[pos + wbase + before] = ((uint32_t)y << 16) | (uint32_t)k;
        pos += total;
        __syncthreads();
    }
}

// energy of the sample-sample bonds of grid blockIdx.y from the stored values, as the compacted
// path's colour kernels would sum it: per colour-1 sample site, its bonds to colour-0 samples,
// c cos + s sin in the compute precision, two-word fixed point.  Sample values are the same in
// every chain, so the grid's first chain is read and the sum is added to each chain's words.
// Blocks take rows (grid-stride), threads plane columns: no element index is divided.
template <class S, class F, bool PER>
__global__ __launch_bounds__(256) void k_econst(const GcDesc* gcs, int n_chains, const void* st,
                                                double q, int64_t* econst)
{
    using St = Store<S>;
    using M = Math<F>;
    __shared__ int64_t sh[4];
    const GcDesc g = gcs[(int64_t)blockIdx.y * n_chains];
    const typename St::raw* p = (const typename St::raw*)st + g.plane_off;
    const int64_t plane = (int64_t)g.H * g.pitch;
    int64_t e_hi = 0, e_lo = 0;
    for (int y = (int)blockIdx.x; y < g.H; y += (int)gridDim.x)
      for (int k = (int)threadIdx.x; 2 * k < g.W; k += (int)blockDim.x) {
        const int x = 2 * k + ((y + 1) & 1);
        if (x >= g.W) continue;
        const typename St::raw v = p[plane + (int64_t)y * g.pitch + k];
        if (!St::sample(v)) continue;
        int xl = x - 1, xr = x + 1, yu = y - 1, yd = y + 1;
        bool el = xl >= 0, er = xr < g.W, eu = yu >= 0, ed = yd < g.H;
        if (PER) {
            xl = el ? xl : xl + g.W; xr = er ? xr : xr - g.W;
            yu = eu ? yu : yu + g.H; yd = ed ? yd : yd - g.H;
            el = er = eu = ed = true;
        }
        F C = (F)0, S_ = (F)0;
        F cs[4], sn[4];
        const int ys[4] = {y, y, yu, yd}, xs[4] = {xl, xr, x, x};
        const bool ex[4] = {el, er, eu, ed};
        for (int n = 0; n < 4; ++n) {
            cs[n] = (F)0; sn[n] = (F)0;
            if (!ex[n]) continue;
            const typename St::raw r = p[(int64_t)ys[n] * g.pitch + (xs[n] >> 1)];
            if (!St::sample(r)) continue;
            M::sincos_rev((F)q * St::template value<F>(r), sn[n], cs[n]);
        }
        C = (cs[0] + cs[1]) + (cs[2] + cs[3]);
        S_ = (sn[0] + sn[1]) + (sn[2] + sn[3]);
        F s0, c0;
        M::sincos_rev((F)q * St::template value<F>(v), s0, c0);
        const Fix2 f = fixed64x2((double)M::fma(c0, C, s0 * S_));
        e_hi += f.hi;
        e_lo += f.lo;
    }
    e_hi = block_sum256(e_hi, sh);
    e_lo = block_sum256(e_lo, sh);
    if (threadIdx.x == 0) {
        for (int ch = 0; ch < n_chains; ++ch) {
            const int64_t gc = (int64_t)blockIdx.y * n_chains + ch;
            atomicAdd((unsigned long long*)&econst[2 * gc], (unsigned long long)e_hi);
            atomicAdd((unsigned long long*)&econst[2 * gc + 1], (unsigned long long)e_lo);
        }
    }
}

// ------------------------------------------------------------------ sweep kernel table
using SweepFn = void (*)(SweepArgs);

template <class S, class F, bool PER> SweepFn pick_sweep_b(int flags, bool esingle)
{
    switch (flags) {
    case 0: return k_sweep<S, F, 0, false, PER>;
    case F_ENERGY: return esingle ? k_sweep<S, F, F_ENERGY, true, PER> : k_sweep<S, F, F_ENERGY, false, PER>;
    case F_ACC: return k_sweep<S, F, F_ACC, false, PER>;
    default: return k_sweep<S, F, F_DEC, false, PER>;
    }
}

template <class S, class F> SweepFn pick_sweep(int flags, bool esingle, bool per)
{
    return per ? pick_sweep_b<S, F, true>(flags, esingle) : pick_sweep_b<S, F, false>(flags, esingle);
}

using SparseFn = void (*)(SparseArgs);

template <class S, class F, bool PER, int C> SparseFn pick_sparse_c(int flags)
{
    switch (flags) {
    case 0: return k_sparse<S, F, 0, PER, C>;
    case F_ENERGY: return k_sparse<S, F, F_ENERGY, PER, C>;
    case F_ACC: return k_sparse<S, F, F_ACC, PER, C>;
    default: return k_sparse<S, F, F_DEC, PER, C>;
    }
}

template <class S, class F> SparseFn pick_sparse(int flags, bool per, int colour)
{
    if (per) return colour ? pick_sparse_c<S, F, true, 1>(flags) : pick_sparse_c<S, F, true, 0>(flags);
    return colour ? pick_sparse_c<S, F, false, 1>(flags) : pick_sparse_c<S, F, false, 0>(flags);
}

using TiledFn = void (*)(TiledArgs);

template <class S, class F, bool PER, int NW, bool TALL> TiledFn pick_tiled_b(int flags)
{
    switch (flags) {
    case 0: return k_tiled<S, F, 0, PER, NW, TALL>;
    case F_ENERGY: return k_tiled<S, F, F_ENERGY, PER, NW, TALL>;
    case F_ACC: return k_tiled<S, F, F_ACC, PER, NW, TALL>;
    default: return k_tiled<S, F, F_DEC, PER, NW, TALL>;
    }
}

template <class S, class F, bool PER> TiledFn pick_tiled_s(int flags, int shape)
{
    // double-precision functions: four-wave blocks on base-height tiles only
    if constexpr (sizeof(F) == 8) {
        return pick_tiled_b<S, F, PER, 4, false>(flags);
    } else {
        switch (shape) {
        case kShapeW8Tall: return pick_tiled_b<S, F, PER, 8, true>(flags);
        case kShapeW4Tall: return pick_tiled_b<S, F, PER, 4, true>(flags);
        case kShapeW8Base: return pick_tiled_b<S, F, PER, 8, false>(flags);
        default: return pick_tiled_b<S, F, PER, 4, false>(flags);
        }
    }
}

template <class S, class F> TiledFn pick_tiled(int flags, bool per, int shape)
{
    return per ? pick_tiled_s<S, F, true>(flags, shape) : pick_tiled_s<S, F, false>(flags, shape);
}

}  // namespace

// ------------------------------------------------------------------ static scratch
// Device memory of mpr_set_temperature_curve_noalloc: the curve table (T, e) and the gathered
// temperatures, in a file-scope array each device holds for the life of the process.  Host code
// never uses the symbol's name as an address: each device's copy lives at its own address,
// looked up once per device (hipGetSymbolAddress with that device current) and kept here.
constexpr int kScratchDoubles = 8192;                 // 64 KiB
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double* g_scratch_ptr[kMaxDevices] = {};

// this device's copy of `scratch` (looked up at the first call on the device)
static hipError_t scratch_address(int device, double** out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = (double*)p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// ------------------------------------------------------------------ context
enum { PH_EMPTY = 0, PH_LOADED = 1, PH_TEMPERED = 2, PH_AVERAGED = 3 };

struct mpr_ctx {
    mpr_config cfg;
    hipStream_t stream = nullptr;
    int device = 0;
    bool broken = false;
    std::string err;
    // shapes
    int G = 0, C = 1;
    std::vector<int64_t> H, W, site_off;      // per grid
    int64_t n_grid_sites = 0;                 // packed per-grid sites
    std::vector<GcDesc> gcs;
    std::vector<Item> items;
    int64_t plane_elems = 0;
    size_t elem = 8;
    int sprec = MPR_FP64;
    bool fsingle = false, esingle = false;
    // device buffers
    GcDesc* d_gcs = nullptr;
    Item* d_items = nullptr;
    GcCtl* d_ctl = nullptr;
    GcCtl* d_ictl = nullptr;     // [2][n_gc] control states during an inference
    int64_t* d_gacc = nullptr;   // [3][n_gc][kAccPerGc] inference accumulators
    RunCtl* d_run = nullptr;
    RunCtl* d_dbg_run = nullptr;
    GridInfo* d_gi = nullptr;
    void* d_state[2] = {nullptr, nullptr};
    double* d_acc = nullptr;     // compact FP64 accumulators: [gc][rank], gc's at its site_off
    uint32_t* d_acc32 = nullptr; // FP16 storage: 32-bit sums of the averaging sweeps since the last
                                 // fold into d_acc (same layout; zero between library calls)
    uint64_t* d_rk_mask = nullptr;   // rank tables of the accumulators (acc_rank)
    int32_t* d_rk_base = nullptr;
    int32_t* d_rk_rows = nullptr;    // per grid and (y, c) row: totals, then their scan
    int64_t* d_rk_row_off = nullptr; // per grid: its first row in d_rk_rows
    int64_t rk_entries = 0, rk_rows = 0, chain_sites = 0;
    double* d_zcopy = nullptr;
    int64_t* d_e_part = nullptr;
    int32_t* d_a_part = nullptr;
    double* d_trace = nullptr;
    int* d_flag = nullptr;
    int64_t trace_cap = 0, trace_len = 0;
    // host mirrors
    std::vector<GridInfo> gi;
    int cur = 0;                 // state buffer holding the current configuration
    int64_t next_sweep = 0, n_avg = 0;
    int phase = PH_EMPTY;
    std::map<std::tuple<int, int, int>, hipGraphExec_t> graphs;   // (mode, cur, length) -> graph
    int graph_k = 0;
    std::vector<int64_t> alloc_sig;                          // shapes the buffers were sized for
    int rows = 16;                                           // rows per work item
    int ctl_threads = 64;                                    // block size of the control kernel
    int64_t item_cap = 0;                                    // items at the smallest row block
    // compacted path (sweep_mode SPARSE): per colour, the prediction-site lists of every grid
    // (shared by its chains) and the waves over them
    bool sparse = false;
    uint32_t* d_sites = nullptr;
    int64_t sites_cap = 0;
    int4* d_waves[2] = {nullptr, nullptr};                   // groups: (gc, first entry, list waves, 0)
    int32_t* d_lead[2] = {nullptr, nullptr};
    int64_t waves_cap[2] = {0, 0};
    int32_t n_waves[2] = {0, 0};                             // groups per colour
    int32_t list_waves[2] = {0, 0};                          // 64-entry list waves per colour
    int32_t group_waves = 1;                                 // list waves per group (at most)
    int64_t list_base0[2] = {0, 0};                          // grid 0's list starts
    int64_t* d_econst = nullptr;                             // [n_gc][2]
    int32_t* d_rowcnt = nullptr;                             // scratch of the list build
    int64_t rowcnt_cap = 0, lead_cap[2] = {0, 0}, econst_cap = 0;
    // LDS-tiled path (sweep_mode TILED): tiles of every (grid, chain), and the sample-sample
    // bond energy (d_econst, shared with the compacted path)
    bool tiled = false;
    int4* d_tiles = nullptr;
    int64_t tiles_cap = 0;
    int32_t n_tiles = 0, tiles_ntx = 0;
    int tile_shape = kShapeW4Base;   // (waves per block, tile height) of the tiled path
    int tile_shape_req = -1;         // shape asked for: forced by the configuration or picked by
                                     // the autotuner; -1 = the automatic rule
    // stream time of the last call of each phase (load, inference / equilibration, averaging,
    // predictions): events recorded before its first and after its last enqueued work
    hipEvent_t ev[4][2] = {};
    bool ev_done[4] = {};
    int64_t ev_sweeps[4] = {};
};

static const char* kStatusText[] = {
    "ok", "invalid argument", "not enough sample data", "periodic grid with an odd side",
    "call out of order", "out of memory", "HIP runtime error",
};

static int fail(mpr_ctx* c, int code, const char* fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
        if (code == MPR_EHIP) c->broken = true;
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, e_ == hipErrorOutOfMemory ? MPR_ENOMEM : MPR_EHIP, "%s: %s",   \
                        #expr, hipGetErrorString(e_));                                      \
    } while (0)

static int check_config(const mpr_config* c)
{
    if (!c) return MPR_EINVAL;
    if (!(c->q > 0.0 && c->q <= 0.5)) return MPR_EINVAL;
    if (!(c->J > 0.0) || !std::isfinite(c->J)) return MPR_EINVAL;
    if (c->precision < MPR_FP64 || c->precision > MPR_FIX16) return MPR_EINVAL;
    if (c->energy_prec < -1 || c->energy_prec > 1 || c->func_prec < -1 || c->func_prec > 1)
        return MPR_EINVAL;
    if ((c->precision == MPR_FP16 || c->precision == MPR_FIX16) && c->func_prec == MPR_PREC_DOUBLE)
        return MPR_EINVAL;
    if (c->boundary != MPR_OPEN && c->boundary != MPR_PERIODIC) return MPR_EINVAL;
    if (c->n_chains < 1) return MPR_EINVAL;
    if (!(c->alpha0 > 0.0 && c->alpha0 <= 1.0)) return MPR_EINVAL;
    if (!(c->acc_target > 0.0 && c->acc_target < 1.0)) return MPR_EINVAL;
    if (!(c->T_min > 0.0) || !(c->T_max >= c->T_min) || !std::isfinite(c->T_max)) return MPR_EINVAL;
    if (c->tile_rows < -1 || c->grid_offset < 0) return MPR_EINVAL;
    if (c->sweep_mode < MPR_SWEEP_AUTO || c->sweep_mode > MPR_SWEEP_TILED) return MPR_EINVAL;
    if (c->tile_shape < 0 || c->tile_shape > kTileShapes) return MPR_EINVAL;
    if (c->group_waves < 0 || c->group_waves > kMaxGroupWaves) return MPR_EINVAL;
    if ((c->sweep_mode == MPR_SWEEP_SPARSE || c->sweep_mode == MPR_SWEEP_TILED) &&
        c->energy_prec == MPR_PREC_SINGLE)
        return MPR_EINVAL;
    return MPR_OK;
}

static void free_device(mpr_ctx* c)
{
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    void* ptrs[] = {c->d_gcs, c->d_items, c->d_ctl, c->d_run, c->d_dbg_run, c->d_gi,
                    c->d_state[0], c->d_state[1], c->d_acc, c->d_acc32, c->d_zcopy, c->d_e_part,
                    c->d_a_part, c->d_trace, c->d_flag, c->d_ictl, c->d_gacc,
                    c->d_rk_mask, c->d_rk_base, c->d_rk_rows, c->d_rk_row_off};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    c->d_gcs = nullptr; c->d_items = nullptr; c->d_ctl = nullptr; c->d_run = nullptr;
    c->d_dbg_run = nullptr; c->d_gi = nullptr; c->d_state[0] = c->d_state[1] = nullptr;
    c->d_acc = nullptr; c->d_acc32 = nullptr; c->d_zcopy = nullptr; c->d_e_part = nullptr; c->d_a_part = nullptr;
    c->d_trace = nullptr; c->d_flag = nullptr; c->d_ictl = nullptr; c->d_gacc = nullptr;
    c->d_rk_mask = nullptr; c->d_rk_base = nullptr; c->d_rk_rows = nullptr; c->d_rk_row_off = nullptr;
    c->trace_cap = 0;
    void* lists[] = {c->d_sites, c->d_waves[0], c->d_waves[1], c->d_lead[0], c->d_lead[1],
                     c->d_econst, c->d_rowcnt, c->d_tiles};
    for (void* p : lists)
        if (p) (void)hipFree(p);
    c->d_sites = nullptr; c->d_waves[0] = c->d_waves[1] = nullptr;
    c->d_lead[0] = c->d_lead[1] = nullptr; c->d_econst = nullptr; c->d_rowcnt = nullptr;
    c->d_tiles = nullptr;
    c->sites_cap = c->waves_cap[0] = c->waves_cap[1] = c->rowcnt_cap = 0;
    c->lead_cap[0] = c->lead_cap[1] = c->econst_cap = c->tiles_cap = 0;
    c->alloc_sig.clear();
}

// Work items: per (grid, chain), row blocks of `rows` rows x strips of 60 lane pairs.  When the
// last strip holds at most 28 pairs (half a wave's output lanes) and `rows` is even, the last
// strips of row blocks b and b + 1 share one two-half item (dy = rows) if every row the two
// blocks read, y0(b) - 2 ... y1(b + 1) + 1, lies inside the grid: row blocks 1, 2 | 3, 4 | ...
// up to the last block that ends at least two rows above the bottom.
static int64_t two_half_items(int64_t np, int64_t H, int rows)
{
    const int64_t last = np - kOutPairs * ((np - 1) / kOutPairs);
    if (rows % 2 || last > kHalfOutPairs) return 0;
    const int64_t inner = (H - 2) / rows - 1;          // blocks 1 ... (H - 2) / rows - 1 qualify
    return inner > 0 ? inner / 2 : 0;
}

static int64_t count_items(const mpr_ctx* c, int rows)
{
    int64_t n = 0;
    for (int g = 0; g < c->G; ++g) {
        const int64_t np = ((c->W[g] + 1) / 2 + 1) / 2;
        const int64_t per = ((np + kOutPairs - 1) / kOutPairs) * ((c->H[g] + rows - 1) / rows);
        n += c->C * (per - two_half_items(np, c->H[g], rows));
    }
    return n;
}

// Heuristic cost of a row-block size: a wave walks rows + 2 colour-0 rows (+ fixed work), and
// the 1024 SIMDs (256 CUs x 4) run the items in ceil(items / 1024) rounds.
static double rows_cost(const mpr_ctx* c, int rows)
{
    const double rounds = std::ceil((double)count_items(c, rows) / 1024.0);
    return rounds * (rows + 3.5);
}

static const int kRowCandidates[] = {2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48,
                                     56, 64, 80, 96, 112, 128, 160, 192, 224, 256};

static int choose_rows(const mpr_ctx* c)
{
    if (c->cfg.tile_rows > 0) return c->cfg.tile_rows;
    // Measured on MI355X: more waves in flight beat longer items until ~32 waves per SIMD
    // (16384^2: 32 rows best), then halo rows cost more than they hide; mid-size grids want
    // >= 4 waves per SIMD (4096^2: 16 rows); grids too small for that use the round model.
    int maxH = 0;
    for (int g = 0; g < c->G; ++g) maxH = std::max<int>(maxH, (int)c->H[g]);
    int best = 0;
    for (int r : kRowCandidates)
        if (r >= 16 && r <= maxH && count_items(c, r) >= 32 * 1024) best = r;
    if (best) return best;
    for (int r : kRowCandidates)
        if (r >= 4 && r <= maxH && count_items(c, r) >= 4 * 1024) best = r;
    if (best) return best;
    best = 4;
    double best_cost = 1e300;
    for (int r : kRowCandidates) {
        if (r > maxH && r > 2) break;
        const double cost = rows_cost(c, r);
        if (cost < best_cost * 0.999) { best_cost = cost; best = r; }
    }
    return best;
}

// work items of every (grid, chain): row blocks of `rows` rows x strips of 60 lane pairs, the
// last strips of pairs of full row blocks in two-half items where they fit (count_items)
static void build_items(mpr_ctx* c, int rows)
{
    c->items.clear();
    int max_items = 1;
    for (size_t i = 0; i < c->gcs.size(); ++i) {
        GcDesc& d = c->gcs[i];
        d.item_begin = (int32_t)c->items.size();
        const int64_t n_two = two_half_items(d.np, d.H, rows);   // blocks 1 ... 2 n_two
        const int last_p0 = kOutPairs * ((d.np - 1) / kOutPairs);
        for (int y0 = 0, b = 0; y0 < d.H; y0 += rows, ++b)
            for (int p0 = 0; p0 < d.np; p0 += kOutPairs) {
                const bool two = p0 == last_p0 && b >= 1 && b <= 2 * n_two;
                if (two && !(b & 1)) continue;                  // swept by block b - 1's item
                c->items.push_back(Item{(int32_t)i, p0, y0, std::min(d.H, y0 + rows), d.plane_off,
                                        d.H, d.W, d.np, d.pitch, two ? rows : 0, 0});
            }
        d.item_end = (int32_t)c->items.size();
        max_items = std::max(max_items, d.item_end - d.item_begin);
    }
    // control kernel: about 8 items per thread, 64 ... 1024 threads
    int t = 64;
    while (t < 1024 && t * 8 < max_items) t *= 2;
    c->ctl_threads = t;
}

static int setup_shapes(mpr_ctx* c, int G, const int64_t* H, const int64_t* W)
{
    if (G < 1) return fail(c, MPR_EINVAL, "n_grids must be >= 1");
    const bool per = c->cfg.boundary == MPR_PERIODIC;
    for (int g = 0; g < G; ++g) {
        if (H[g] < 2 || W[g] < 2) return fail(c, MPR_EINVAL, "grid %d: sides must be >= 2", g);
        if (H[g] > (1 << 30) || W[g] > (1 << 30) || H[g] * W[g] > (int64_t)1 << 40)
            return fail(c, MPR_EINVAL, "grid %d: too large", g);
        if (per && ((H[g] & 1) || (W[g] & 1)))
            return fail(c, MPR_EBIPARTITE, "grid %d: periodic boundary needs even sides", g);
        if (per && (W[g] % 4))
            return fail(c, MPR_EINVAL, "grid %d: periodic boundary needs W divisible by 4", g);
        const int64_t np = ((W[g] + 1) / 2 + 1) / 2;
        const int64_t pitch = ((2 * np + 63) / 64) * 64;
        // the sweep addresses a (grid, chain)'s two planes of FP64 accumulators through one
        // buffer resource of at most kBufMaxBytes
        if (2 * H[g] * pitch * (int64_t)sizeof(double) > (int64_t)kBufMaxBytes)
            return fail(c, MPR_EINVAL, "grid %d: too large (2 H pitch 8 bytes > %u)", g, kBufMaxBytes);
    }
    c->G = G;
    c->C = c->cfg.n_chains;
    c->H.assign(H, H + G);
    c->W.assign(W, W + G);
    c->site_off.resize(G);
    int64_t off = 0;
    for (int g = 0; g < G; ++g) { c->site_off[g] = off; off += H[g] * W[g]; }
    c->n_grid_sites = off;
    c->gcs.clear();
    int64_t plane = 0, rk = 0, rk_rows = 0;
    for (int g = 0; g < G; ++g) {
        const int64_t np_g = ((W[g] + 1) / 2 + 1) / 2, pitch_g = ((2 * np_g + 63) / 64) * 64;
        const int64_t rk_g = rk;
        rk += 2 * H[g] * (pitch_g / 64);
        rk_rows += 2 * H[g];
        for (int ch = 0; ch < c->C; ++ch) {
            GcDesc d{};
            d.H = (int32_t)H[g];
            d.W = (int32_t)W[g];
            d.wc = (int32_t)((W[g] + 1) / 2);
            d.np = (d.wc + 1) / 2;
            d.pitch = ((2 * d.np + 63) / 64) * 64;
            d.chain_word = (c->cfg.grid_offset + g) * c->C + ch;
            d.grid = g;
            d.plane_off = plane;
            plane += 2 * (int64_t)d.H * d.pitch;
            d.grid_site_off = c->site_off[g];
            d.n_bonds = per ? 2 * H[g] * W[g] : 2 * H[g] * W[g] - H[g] - W[g];
            d.inv_n_bonds = d.n_bonds > 0 ? 1.0 / (double)d.n_bonds : 0.0;
            d.rk_off = rk_g;
            c->gcs.push_back(d);
        }
    }
    c->rk_entries = rk;
    c->rk_rows = rk_rows;
    c->rows = choose_rows(c);
    build_items(c, c->rows);
    const int rmin = std::min(c->rows, 2);
    c->item_cap = 0;
    for (const auto& d : c->gcs)
        c->item_cap += (int64_t)((d.np + kOutPairs - 1) / kOutPairs) * ((d.H + rmin - 1) / rmin);
    // per-chain packed site offsets: [g][chain][H*W]
    int64_t so = 0;
    for (int g = 0; g < G; ++g)
        for (int ch = 0; ch < c->C; ++ch) { c->gcs[g * c->C + ch].site_off = so; so += H[g] * W[g]; }
    c->chain_sites = so;
    c->plane_elems = plane;
    return MPR_OK;
}

// host -> device copy ordered on the context's stream (the caller's stream may be a
// non-blocking stream, which a plain hipMemcpy on the null stream would not wait for); the
// stream is synchronised so the host buffer may be released right after
static hipError_t h2d(mpr_ctx* c, void* dst, const void* src, size_t bytes)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c->stream);
}

static int alloc_device(mpr_ctx* c)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const size_t n_gc = c->gcs.size(), n_items = c->items.size();
    // a reload with the same shapes reuses every buffer (and the captured graphs)
    std::vector<int64_t> sig = {(int64_t)n_gc, (int64_t)n_items, c->plane_elems, c->n_grid_sites, c->rows};
    for (int g = 0; g < c->G; ++g) { sig.push_back(c->H[g]); sig.push_back(c->W[g]); }
    if (c->d_gcs && sig == c->alloc_sig) {
        HIPCHK(c, h2d(c, c->d_gcs, c->gcs.data(), n_gc * sizeof(GcDesc)));
        RunCtl r{0, 0, 0, 0};
        HIPCHK(c, h2d(c, c->d_run, &r, sizeof r));
        return MPR_OK;
    }
    free_device(c);
    c->alloc_sig = sig;
    HIPCHK(c, hipMalloc(&c->d_gcs, n_gc * sizeof(GcDesc)));
    HIPCHK(c, hipMalloc(&c->d_items, c->item_cap * sizeof(Item)));
    HIPCHK(c, hipMalloc(&c->d_ctl, n_gc * sizeof(GcCtl)));
    HIPCHK(c, hipMalloc(&c->d_ictl, 2 * n_gc * sizeof(GcCtl)));
    HIPCHK(c, hipMalloc(&c->d_gacc, 3 * n_gc * kAccPerGc * sizeof(int64_t)));
    HIPCHK(c, hipMalloc(&c->d_run, sizeof(RunCtl)));
    HIPCHK(c, hipMalloc(&c->d_dbg_run, sizeof(RunCtl)));
    HIPCHK(c, hipMalloc(&c->d_gi, c->G * sizeof(GridInfo)));
    for (int b = 0; b < 2; ++b) HIPCHK(c, hipMalloc(&c->d_state[b], c->plane_elems * c->elem));
    HIPCHK(c, hipMalloc(&c->d_acc, c->chain_sites * sizeof(double)));
    if (c->sprec == MPR_FP16) HIPCHK(c, hipMalloc(&c->d_acc32, c->chain_sites * sizeof(uint32_t)));
    HIPCHK(c, hipMalloc(&c->d_rk_mask, std::max<int64_t>(c->rk_entries, 1) * sizeof(uint64_t)));
    HIPCHK(c, hipMalloc(&c->d_rk_base, std::max<int64_t>(c->rk_entries, 1) * sizeof(int32_t)));
    HIPCHK(c, hipMalloc(&c->d_rk_rows, std::max<int64_t>(c->rk_rows, 1) * sizeof(int32_t)));
    HIPCHK(c, hipMalloc(&c->d_rk_row_off, c->G * sizeof(int64_t)));
    {
        std::vector<int64_t> ro(c->G);
        int64_t r = 0;
        for (int g = 0; g < c->G; ++g) { ro[g] = r; r += 2 * c->H[g]; }
        HIPCHK(c, h2d(c, c->d_rk_row_off, ro.data(), c->G * sizeof(int64_t)));
    }
    HIPCHK(c, hipMalloc(&c->d_zcopy, c->n_grid_sites * sizeof(double)));
    HIPCHK(c, hipMalloc(&c->d_e_part, 2 * c->item_cap * sizeof(int64_t)));
    HIPCHK(c, hipMalloc(&c->d_a_part, c->item_cap * sizeof(int32_t)));
    HIPCHK(c, hipMalloc(&c->d_flag, sizeof(int)));
    HIPCHK(c, h2d(c, c->d_gcs, c->gcs.data(), n_gc * sizeof(GcDesc)));
    HIPCHK(c, h2d(c, c->d_items, c->items.data(), n_items * sizeof(Item)));
    RunCtl r{0, 0, 0, 0};
    HIPCHK(c, h2d(c, c->d_run, &r, sizeof r));
    HIPCHK(c, h2d(c, c->d_dbg_run, &r, sizeof r));
    return MPR_OK;
}

static dim3 site_grid(int64_t n, int ys, int64_t max_blocks = 4096)
{
    int64_t b = (n + 255) / 256;
    b = std::max<int64_t>(1, std::min<int64_t>(b, max_blocks));
    return dim3((unsigned)b, (unsigned)ys);
}

template <class S> static void launch_map(mpr_ctx* c, const double* z, const uint8_t* mask)
{
    int64_t maxp = 0;
    for (auto& g : c->gcs) maxp = std::max<int64_t>(maxp, 2 * (int64_t)g.H * g.pitch);
    const uint32_t k0 = (uint32_t)(c->cfg.seed & 0xffffffffu), k1 = (uint32_t)(c->cfg.seed >> 32);
    hipLaunchKernelGGL(k_map_init<S>, site_grid(maxp, (int)c->gcs.size()), dim3(256), 0, c->stream,
                       c->d_gcs, c->d_gi, z, mask, c->d_state[0], c->d_state[1],
                       k0, k1);
}

template <class S> static void launch_get_state(mpr_ctx* c, double* u, double* acc, dim3 grid)
{
    hipLaunchKernelGGL(k_get_state<S>, grid, dim3(256), 0, c->stream, c->d_gcs, c->d_state[c->cur], c->d_acc, c->d_rk_mask, c->d_rk_base, u, acc);
}
template <class S> static void launch_set_state(mpr_ctx* c, const double* u, const double* acc, int mode, dim3 grid)
{
    hipLaunchKernelGGL(k_set_state<S>, grid, dim3(256), 0, c->stream, c->d_gcs, c->d_state[c->cur], c->d_acc, c->d_rk_mask, c->d_rk_base, u, acc, c->d_flag, mode);
}

// grow a device buffer to at least `bytes` (contents dropped); captured graphs hold the old
// address, so they are dropped too
static int ensure_buffer(mpr_ctx* c, void** p, int64_t* cap, int64_t bytes)
{
    if (*p && *cap >= bytes) return MPR_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    HIPCHK(c, hipMalloc(p, (size_t)std::max<int64_t>(bytes, 256)));
    *cap = bytes;
    return MPR_OK;
}

template <class S> static void launch_list_count(mpr_ctx* c, int hmax, const int64_t* row_off)
{
    hipLaunchKernelGGL(k_list_count<S>, dim3(hmax, 2 * c->G), dim3(256), 0, c->stream, c->d_gcs, c->C,
                       c->d_state[c->cur], c->d_rowcnt, row_off);
}

template <class S>
static void launch_list_fill(mpr_ctx* c, int hmax, const int64_t* row_off, const int64_t* base)
{
    hipLaunchKernelGGL(k_list_fill<S>, dim3(hmax, 2 * c->G), dim3(256), 0, c->stream, c->d_gcs, c->C,
                       c->d_state[c->cur], c->d_rowcnt, row_off, base, c->d_sites);
}

template <class S, class F> static void launch_econst(mpr_ctx* c)
{
    int hmax = 1;
    for (int g = 0; g < c->G; ++g) hmax = std::max<int>(hmax, (int)c->H[g]);
    const dim3 grid((unsigned)std::min(hmax, 1024), (unsigned)c->G);   // rows x grids
    auto fn = c->cfg.boundary == MPR_PERIODIC ? k_econst<S, F, true> : k_econst<S, F, false>;
    hipLaunchKernelGGL(fn, grid, dim3(256), 0, c->stream, c->d_gcs, c->C, c->d_state[c->cur], c->cfg.q,
                       c->d_econst);
}

static int build_econst(mpr_ctx* c);

// tiles of the tiled path: per (grid, chain), row blocks of the tile height x column blocks of
// kTileCols plane columns, row-major (neighbouring tiles get neighbouring block numbers).  The
// shape: forced by the configuration or chosen by the autotuner (shape >= 0), else the rule --
// with single-precision functions and fewer than kTileWavesSwitch tiles of the base height,
// eight-wave blocks on tiles of twice that height; else four-wave blocks on base-height tiles.
template <class S, class F> static int build_tiles_t(mpr_ctx* c, int shape)
{
    int64_t base = 0;
    for (const GcDesc& d : c->gcs)
        base += (int64_t)((d.H + tile_rows<S, F>() - 1) / tile_rows<S, F>()) * ((d.wc + kTileCols - 1) / kTileCols);
    if (sizeof(F) == 8) shape = kShapeW4Base;
    else if (shape < 0) shape = base < kTileWavesSwitch ? kShapeW8Tall : kShapeW4Base;
    c->tile_shape = shape;
    const int TY = shape_tall(shape) ? tile_rows_for<S, F, true>() : tile_rows_for<S, F, false>();
    std::vector<int4> t;
    for (int i = 0; i < (int)c->gcs.size(); ++i) {
        const GcDesc& d = c->gcs[i];
        const int nty = (d.H + TY - 1) / TY, ntx = (d.wc + kTileCols - 1) / kTileCols;
        if (i == 0) c->tiles_ntx = ntx;
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx)
                t.push_back(int4{i, ty * TY, tx * kTileCols, (ty == 0 && tx == 0) ? 1 : 0});
        if (t.size() > (size_t)INT32_MAX) return fail(c, MPR_EINVAL, "too many tiles");
    }
    c->n_tiles = (int32_t)t.size();
    if (c->gcs.size() > 1) {
        int rc = ensure_buffer(c, (void**)&c->d_tiles, &c->tiles_cap, (int64_t)t.size() * sizeof(int4));
        if (rc) return rc;
        HIPCHK(c, h2d(c, c->d_tiles, t.data(), t.size() * sizeof(int4)));
    }
    return build_econst(c);
}

static int build_tiles(mpr_ctx* c, int shape)
{
    switch (c->sprec) {
    case MPR_FP64: return c->fsingle ? build_tiles_t<double, float>(c, shape) : build_tiles_t<double, double>(c, shape);
    case MPR_FP32: return c->fsingle ? build_tiles_t<float, float>(c, shape) : build_tiles_t<float, double>(c, shape);
    case MPR_FIX16: return build_tiles_t<Fix15, float>(c, shape);
    default: return build_tiles_t<_Float16, float>(c, shape);
    }
}

// prediction-site lists of the compacted path, their waves, and the sample-sample bond energy
static int build_lists(mpr_ctx* c)
{
    const int G = c->G, C = c->C, n_gc = (int)c->gcs.size();
    std::vector<int64_t> meta(3 * G);                  // row offsets [G], list bases [2G]
    int64_t rows = 0;
    int hmax = 0;
    for (int g = 0; g < G; ++g) {
        meta[g] = rows;
        rows += 2 * c->H[g];
        hmax = std::max<int>(hmax, (int)c->H[g]);
    }
    // scratch: row counts [rows] | totals [2G] | meta (int64) [3G]
    const int64_t meta_at = ((rows + 2 * G) * 4 + 7) / 8 * 8;
    int rc = ensure_buffer(c, (void**)&c->d_rowcnt, &c->rowcnt_cap, meta_at + 3 * G * 8);
    if (rc) return rc;
    int32_t* d_tot = c->d_rowcnt + rows;
    int64_t* d_meta = (int64_t*)((char*)c->d_rowcnt + meta_at);
    HIPCHK(c, h2d(c, d_meta, meta.data(), G * sizeof(int64_t)));
    switch (c->sprec) {
    case MPR_FP64: launch_list_count<double>(c, hmax, d_meta); break;
    case MPR_FP32: launch_list_count<float>(c, hmax, d_meta); break;
    case MPR_FIX16: launch_list_count<Fix15>(c, hmax, d_meta); break;
    default: launch_list_count<_Float16>(c, hmax, d_meta); break;
    }
    hipLaunchKernelGGL(k_list_scan, dim3(2 * G), dim3(256), 0, c->stream, c->d_gcs, C, c->d_rowcnt, d_meta, d_tot);
    HIPCHK(c, hipGetLastError());
    std::vector<int32_t> tot(2 * G);
    HIPCHK(c, hipMemcpyAsync(tot.data(), d_tot, 2 * G * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // lists padded to whole waves (at least one per grid and colour, so every (grid, chain) has
    // a lead wave in both launches)
    int64_t entries = 0;
    for (int i = 0; i < 2 * G; ++i) {
        meta[G + i] = entries;
        entries += std::max<int64_t>(1, (tot[i] + kWave - 1) / kWave) * kWave;
    }
    // A compacted-path wave sweeps a group of up to group_waves consecutive list waves of one
    // (grid, chain), so the per-wave work (control step, reductions, atomics, the first loads)
    // is shared by up to group_waves x 64 sites; groups stay numerous enough to fill the chip
    // (about 20 480 per colour, two and a half rounds of eight resident waves per SIMD) before
    // they grow (measured on the 256-grid batch in FP16: 4, 8, 16, 32, 64, 128 list waves per
    // group gave 1.205, 1.024, 0.942, 0.917, 0.934, 0.968 ms per sweep).
    int64_t lw_total = 0;
    for (int i = 0; i < n_gc; ++i)
        for (int col = 0; col < 2; ++col)
            lw_total += std::max<int64_t>(1, ((int64_t)tot[2 * c->gcs[i].grid + col] + kWave - 1) / kWave);
    const int ns = c->cfg.group_waves > 0
                       ? c->cfg.group_waves
                       : (int)std::min<int64_t>(kMaxGroupWaves, std::max<int64_t>(1, lw_total / 2 / kGroupTarget));
    std::vector<int4> waves[2];
    std::vector<int32_t> lead[2];
    int32_t list_waves[2] = {0, 0};
    for (int col = 0; col < 2; ++col) {
        lead[col].resize(n_gc);
        for (int i = 0; i < n_gc; ++i) {
            const int gr = c->gcs[i].grid;
            const int64_t nw = std::max<int64_t>(1, ((int64_t)tot[2 * gr + col] + kWave - 1) / kWave);
            lead[col][i] = (int32_t)waves[col].size();
            for (int64_t w = 0; w < nw; w += ns)
                waves[col].push_back(int4{i, (int)(meta[G + 2 * gr + col] + w * kWave),
                                          (int)std::min<int64_t>(ns, nw - w), 0});
            if (i == 0) list_waves[col] = (int32_t)std::min<int64_t>(nw, INT32_MAX);
        }
        if (waves[col].size() > (size_t)INT32_MAX / kWavesPerBlock)
            return fail(c, MPR_EINVAL, "too many prediction sites for the compacted path");
    }
    if (entries > (int64_t)INT32_MAX) return fail(c, MPR_EINVAL, "too many prediction sites for the compacted path");
    // captured sweeps hold the wave counts and list bases in their arguments: a reload with the
    // same shapes but other lists must capture again
    if (meta[G] != c->list_base0[0] || meta[G + 1] != c->list_base0[1] ||
        (int64_t)waves[0].size() != c->n_waves[0] || (int64_t)waves[1].size() != c->n_waves[1] ||
        ns != c->group_waves || list_waves[0] != c->list_waves[0] || list_waves[1] != c->list_waves[1]) {
        for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
        c->graphs.clear();
    }
    c->list_base0[0] = meta[G];
    c->list_base0[1] = meta[G + 1];
    c->group_waves = ns;
    c->list_waves[0] = list_waves[0];
    c->list_waves[1] = list_waves[1];
    rc = ensure_buffer(c, (void**)&c->d_sites, &c->sites_cap, entries * 4);
    if (rc) return rc;
    HIPCHK(c, hipMemsetAsync(c->d_sites, 0xff, entries * 4, c->stream));
    HIPCHK(c, h2d(c, d_meta + G, meta.data() + G, 2 * G * sizeof(int64_t)));
    switch (c->sprec) {
    case MPR_FP64: launch_list_fill<double>(c, hmax, d_meta, d_meta + G); break;
    case MPR_FP32: launch_list_fill<float>(c, hmax, d_meta, d_meta + G); break;
    case MPR_FIX16: launch_list_fill<Fix15>(c, hmax, d_meta, d_meta + G); break;
    default: launch_list_fill<_Float16>(c, hmax, d_meta, d_meta + G); break;
    }
    for (int col = 0; col < 2; ++col) {
        c->n_waves[col] = (int32_t)waves[col].size();
        rc = ensure_buffer(c, (void**)&c->d_waves[col], &c->waves_cap[col], (int64_t)waves[col].size() * sizeof(int4));
        if (rc) return rc;
        rc = ensure_buffer(c, (void**)&c->d_lead[col], &c->lead_cap[col], (int64_t)n_gc * sizeof(int32_t));
        if (rc) return rc;
        HIPCHK(c, h2d(c, c->d_waves[col], waves[col].data(), waves[col].size() * sizeof(int4)));
        HIPCHK(c, h2d(c, c->d_lead[col], lead[col].data(), n_gc * sizeof(int32_t)));
    }
    return build_econst(c);
}

// sample-sample bond energy per (grid, chain): seeds the accumulators of the compacted and
// tiled paths, whose sweeps sum only bonds that touch a prediction site
static int build_econst(mpr_ctx* c)
{
    const int n_gc = (int)c->gcs.size();
    int rc = ensure_buffer(c, (void**)&c->d_econst, &c->econst_cap, 2 * (int64_t)n_gc * sizeof(int64_t));
    if (rc) return rc;
    HIPCHK(c, hipMemsetAsync(c->d_econst, 0, 2 * n_gc * sizeof(int64_t), c->stream));
    switch (c->sprec) {
    case MPR_FP64: if (c->fsingle) launch_econst<double, float>(c); else launch_econst<double, double>(c); break;
    case MPR_FP32: if (c->fsingle) launch_econst<float, float>(c); else launch_econst<float, double>(c); break;
    case MPR_FIX16: launch_econst<Fix15, float>(c); break;
    default: launch_econst<_Float16, float>(c); break;
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));      // host tables above go out of scope
    return MPR_OK;
}

// whether the compacted path can run this context (double-precision energy, 16-bit list
// coordinates) and the tiled path (double-precision energy)
static bool sparse_possible(const mpr_ctx* c)
{
    bool possible = !c->esingle;
    for (int g = 0; g < c->G; ++g) {
        const GcDesc& d = c->gcs[(size_t)g * c->C];
        possible = possible && d.H < 65536 && d.pitch < 65536;
    }
    return possible;
}
static bool tiled_possible(const mpr_ctx* c) { return !c->esingle; }

// the automatic rule (measured crossovers, see include/mpr.h)
static int auto_path(const mpr_ctx* c)
{
    int64_t P = 0, N = 0;
    for (int g = 0; g < c->G; ++g) {
        P += c->gi[g].n_pred;
        N += c->H[g] * c->W[g];
    }
    const double frac = (double)P / (double)N, work = (double)N * c->C;
    // the tiled path wins where a sweep is latency-bound (one launch per sweep instead of two,
    // no list reads): small grids with single-precision functions, and with double-precision
    // functions once most sites are prediction sites
    if (tiled_possible(c) && work <= 1572864.0 && (c->fsingle || frac > 0.6)) return MPR_SWEEP_TILED;
    // the compacted path in groups: with 16-bit storage it beats the fused kernel once half the
    // sites or fewer are prediction sites (batch of 256 grids at 43 %: 0.93 against 1.19 ms per
    // sweep; 16384^2 at 50 %: 0.72 against 0.75 ms); with double-precision functions up to 60 %
    // at any size; with FP32 storage its doubled bytes stall it beyond small grids
    const bool prefer = c->fsingle ? (c->elem == 2 ? frac <= 0.5 : (frac <= 0.4 && work <= 8388608.0))
                                   : (frac <= 0.6 || (frac <= 0.7 && work <= 8388608.0));
    return (sparse_possible(c) && prefer) ? MPR_SWEEP_SPARSE : MPR_SWEEP_FUSED;
}

// switch the context to sweep path `path` (lists or tiles built for the loaded data)
static int apply_path(mpr_ctx* c, int path)
{
    const bool sparse = path == MPR_SWEEP_SPARSE, tiled = path == MPR_SWEEP_TILED;
    if (sparse != c->sparse || tiled != c->tiled) {   // graphs hold the other path's kernels
        for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
        c->graphs.clear();
    }
    c->sparse = sparse;
    c->tiled = tiled;
    return sparse ? build_lists(c) : (tiled ? build_tiles(c, c->tile_shape_req) : MPR_OK);
}

// the sweep path for the loaded data (sweep_mode, or the automatic rule)
static int choose_path(mpr_ctx* c)
{
    const int mode = c->cfg.sweep_mode;
    if (mode == MPR_SWEEP_SPARSE && !sparse_possible(c))
        return fail(c, MPR_EINVAL, "the compacted sweep needs double-precision energy and sides below 65536");
    if (mode == MPR_SWEEP_TILED && !tiled_possible(c))
        return fail(c, MPR_EINVAL, "the tiled sweep needs double-precision energy");
    return apply_path(c, mode == MPR_SWEEP_AUTO ? auto_path(c) : mode);
}

static int current_path(const mpr_ctx* c)
{
    return c->sparse ? MPR_SWEEP_SPARSE : (c->tiled ? MPR_SWEEP_TILED : MPR_SWEEP_FUSED);
}

extern "C" {

void mpr_config_default(mpr_config* cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->q = 0.5;
    cfg->J = 1.0;
    cfg->precision = MPR_FP64;
    cfg->energy_prec = MPR_PREC_DEFAULT;
    cfg->func_prec = MPR_PREC_DEFAULT;
    cfg->boundary = MPR_OPEN;
    cfg->n_chains = 1;
    cfg->seed = 1;
    cfg->alpha0 = 1.0;
    cfg->acc_target = 0.3;
    cfg->T_min = 1e-6;
    cfg->T_max = 10.0;
}

const char* mpr_strerror(int s)
{
    if (s < 0 || s > MPR_EHIP) return "unknown status";
    return kStatusText[s];
}

const char* mpr_last_error(mpr_ctx* c) { return c ? c->err.c_str() : "null context"; }

static int create_common(const mpr_config* cfg, void* stream, mpr_ctx** out)
{
    if (!out) return MPR_EINVAL;
    *out = nullptr;
    int rc = check_config(cfg);
    if (rc) return rc;
    mpr_ctx* c = new (std::nothrow) mpr_ctx();
    if (!c) return MPR_ENOMEM;
    c->cfg = *cfg;
    c->stream = (hipStream_t)stream;
    c->sprec = cfg->precision;
    c->elem = cfg->precision == MPR_FP64 ? 8 : (cfg->precision == MPR_FP32 ? 4 : 2);   // FP16, FIX16: 2
    c->fsingle = cfg->func_prec == MPR_PREC_DEFAULT ? cfg->precision != MPR_FP64
                                                    : cfg->func_prec == MPR_PREC_SINGLE;
    c->esingle = cfg->energy_prec == MPR_PREC_SINGLE;
    if (cfg->tile_shape > 0) {   // a forced tile shape; the eight-wave and tall ones need single-precision functions
        if (!c->fsingle && cfg->tile_shape - 1 != kShapeW4Base) { delete c; return MPR_EINVAL; }
        c->tile_shape_req = cfg->tile_shape - 1;
    }
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return MPR_EHIP; }
    c->graph_k = cfg->graph_sweeps == 0 ? 32 : cfg->graph_sweeps;
    if (c->graph_k > 0 && (c->graph_k & 1)) c->graph_k += 1;
    if (!c->stream) c->graph_k = -1;   // the legacy default stream cannot be captured
    *out = c;
    return MPR_OK;
}

int mpr_create(const mpr_config* cfg, void* stream, mpr_ctx** out)
{
    return create_common(cfg, stream, out);
}

int mpr_batch_create(const mpr_config* cfg, void* stream, int32_t n_grids, const int64_t* H,
                     const int64_t* W, mpr_ctx** out)
{
    if (!H || !W || n_grids < 1) return MPR_EINVAL;
    int rc = create_common(cfg, stream, out);
    if (rc) return rc;
    rc = setup_shapes(*out, n_grids, H, W);
    if (rc) { delete *out; *out = nullptr; }
    return rc;
}

void mpr_destroy(mpr_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    free_device(c);
    for (auto& pair : c->ev)
        for (hipEvent_t e : pair)
            if (e) (void)hipEventDestroy(e);
    delete c;
}

enum { PHASE_LOAD = 0, PHASE_INFER = 1, PHASE_RUN = 2, PHASE_PREDICT = 3 };

// records the start (end = 0) or the end (end = 1) of a phase on the context's stream
static int mark(mpr_ctx* c, int phase, int end, int64_t sweeps = 0)
{
    hipEvent_t& e = c->ev[phase][end];
    if (!e) HIPCHK(c, hipEventCreate(&e));
    HIPCHK(c, hipEventRecord(e, c->stream));
    if (end) { c->ev_done[phase] = true; c->ev_sweeps[phase] = sweeps; }
    else c->ev_done[phase] = false;
    return MPR_OK;
}

static int usable(mpr_ctx* c)
{
    if (!c) return MPR_EINVAL;
    if (c->broken) return fail(c, MPR_EHIP, "context is unusable after an earlier HIP error");
    return MPR_OK;
}

static int autotune(mpr_ctx* c, int n, int* best_out);

// free_only: a lattice with no data at all (the unconditional model of the energy curve)
static int load_common(mpr_ctx* c, const double* z, const uint8_t* mask, bool free_only = false)
{
    int rc = alloc_device(c);
    if (rc) return rc;
    rc = mark(c, PHASE_LOAD, 0);
    if (rc) return rc;
    c->gi.assign(c->G, GridInfo{});
    int64_t max_sites = 0;
    for (int g = 0; g < c->G; ++g) {
        GridInfo& G = c->gi[g];
        G.H = c->H[g]; G.W = c->W[g]; G.site_off = c->site_off[g];
        G.min_ord = ~0ull; G.max_ord = 0;
        max_sites = std::max(max_sites, G.H * G.W);
    }
    HIPCHK(c, hipMemcpyAsync(c->d_gi, c->gi.data(), c->G * sizeof(GridInfo), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_scan, site_grid(max_sites, c->G, 256), dim3(256), 0, c->stream, c->d_gi, z, mask);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->gi.data(), c->d_gi, c->G * sizeof(GridInfo), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int g = 0; g < c->G && !free_only; ++g) {
        GridInfo& G = c->gi[g];
        if (G.flags & 1) return fail(c, MPR_EINVAL, "grid %d: mask values must be 0 or 1", g);
        if (G.flags & 2) return fail(c, MPR_EINVAL, "grid %d: non-finite value at a sample site", g);
        if (G.n_sample < 1) return fail(c, MPR_ENOSAMPLE, "grid %d: no sample site", g);
        G.zmin = order_inverse(G.min_ord);
        G.zmax = order_inverse(G.max_ord);
        if (!(G.zmax > G.zmin)) return fail(c, MPR_ENOSAMPLE, "grid %d: all sample values are equal", g);
    }
    HIPCHK(c, hipMemcpyAsync(c->d_gi, c->gi.data(), c->G * sizeof(GridInfo), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_sample_energy, site_grid(max_sites, c->G, 256), dim3(256), 0, c->stream, c->d_gi,
                       z, mask, c->cfg.q, (int)(c->cfg.boundary == MPR_PERIODIC));
    hipLaunchKernelGGL(k_copy_z, site_grid(max_sites, c->G), dim3(256), 0, c->stream, c->d_gi, z, c->d_zcopy);
    switch (c->sprec) {
    case MPR_FP64: launch_map<double>(c, z, mask); break;
    case MPR_FP32: launch_map<float>(c, z, mask); break;
    case MPR_FIX16: launch_map<Fix15>(c, z, mask); break;
    default: launch_map<_Float16>(c, z, mask); break;
    }
    HIPCHK(c, hipGetLastError());
    // compact accumulators: zeroed, and the rank tables of this data's prediction sites
    HIPCHK(c, hipMemsetAsync(c->d_acc, 0, c->chain_sites * sizeof(double), c->stream));
    if (c->d_acc32) HIPCHK(c, hipMemsetAsync(c->d_acc32, 0, c->chain_sites * sizeof(uint32_t), c->stream));
    {
        int64_t max_e = 0, max_rows = 0;
        for (int g = 0; g < c->G; ++g) {
            const GcDesc& d = c->gcs[(size_t)g * c->C];
            max_e = std::max<int64_t>(max_e, 2 * (int64_t)d.H * (d.pitch / 64));
            max_rows = std::max<int64_t>(max_rows, 2 * (int64_t)d.H);
        }
        hipLaunchKernelGGL(k_rank_count, site_grid(max_e, c->G, 1024), dim3(256), 0, c->stream, c->d_gcs, c->C,
                           mask, c->d_rk_mask, c->d_rk_base);
        hipLaunchKernelGGL(k_rank_rows, site_grid(max_rows, c->G, 64), dim3(256), 0, c->stream, c->d_gcs, c->C,
                           c->d_rk_base, c->d_rk_rows, c->d_rk_row_off);
        hipLaunchKernelGGL(k_rank_rowscan, dim3((unsigned)c->G), dim3(256), 0, c->stream, c->d_gcs, c->C,
                           c->d_rk_rows, c->d_rk_row_off);
        hipLaunchKernelGGL(k_rank_add, site_grid(max_e, c->G, 1024), dim3(256), 0, c->stream, c->d_gcs, c->C,
                           c->d_rk_base, c->d_rk_rows, c->d_rk_row_off);
        HIPCHK(c, hipGetLastError());
    }
    HIPCHK(c, hipMemcpyAsync(c->gi.data(), c->d_gi, c->G * sizeof(GridInfo), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<GcCtl> ctl(c->gcs.size());
    for (size_t i = 0; i < c->gcs.size(); ++i) {
        GcDesc& d = c->gcs[i];
        const GridInfo& G = c->gi[d.grid];
        if (G.n_sample_bonds == 0 && !free_only)
            return fail(c, MPR_ENOSAMPLE, "grid %d: no bond joins two sample sites", d.grid);
        d.n_pred = G.n_pred;
        d.inv_n_pred = G.n_pred > 0 ? 1.0 / (double)G.n_pred : 0.0;
        GcCtl& k = ctl[i];
        std::memset(&k, 0, sizeof k);
        k.alpha = c->cfg.alpha0;
        k.e_smp = free_only ? 0.0 : -c->cfg.J * fix2_value(G.e_hi, G.e_lo) / (double)G.n_sample_bonds;
    }
    HIPCHK(c, h2d(c, c->d_gcs, c->gcs.data(), c->gcs.size() * sizeof(GcDesc)));
    HIPCHK(c, h2d(c, c->d_ctl, ctl.data(), ctl.size() * sizeof(GcCtl)));
    c->cur = 0;
    c->next_sweep = 0;
    c->n_avg = 0;
    c->trace_len = 0;
    int prc = choose_path(c);
    if (prc) return prc;
    c->phase = PH_LOADED;
    if (c->cfg.tile_rows == -1) {
        const int trc = autotune(c, 8, nullptr);
        if (trc) return trc;
    }
    return mark(c, PHASE_LOAD, 1);
}

int mpr_load(mpr_ctx* c, int64_t H, int64_t W, const double* z, const uint8_t* mask)
{
    int rc = usable(c);
    if (rc) return rc;
    if (!z || !mask) return fail(c, MPR_EINVAL, "null data pointer");
    if (c->G > 1) return fail(c, MPR_EINVAL, "batched context: use mpr_batch_load");
    rc = setup_shapes(c, 1, &H, &W);
    if (rc) { c->phase = PH_EMPTY; return rc; }
    rc = load_common(c, z, mask);
    if (rc) c->phase = PH_EMPTY;
    return rc;
}

int mpr_batch_load(mpr_ctx* c, const double* z, const uint8_t* mask)
{
    int rc = usable(c);
    if (rc) return rc;
    if (!z || !mask) return fail(c, MPR_EINVAL, "null data pointer");
    if (c->G < 1) return fail(c, MPR_ESTATE, "no grid shapes: use mpr_load or mpr_batch_create");
    rc = load_common(c, z, mask);
    if (rc) c->phase = PH_EMPTY;
    return rc;
}

// ------------------------------------------------------------------ sweep launches
enum { MODE_EQUIL = 0, MODE_AVG = 1, MODE_BURN = 2 };

static SweepFn sweep_fn(const mpr_ctx* c, int flags)
{
    const bool per = c->cfg.boundary == MPR_PERIODIC;
    switch (c->sprec) {
    case MPR_FP64: return c->fsingle ? pick_sweep<double, float>(flags, c->esingle, per)
                                     : pick_sweep<double, double>(flags, c->esingle, per);
    case MPR_FP32: return c->fsingle ? pick_sweep<float, float>(flags, c->esingle, per)
                                     : pick_sweep<float, double>(flags, c->esingle, per);
    case MPR_FIX16: return pick_sweep<Fix15, float>(flags, c->esingle, per);
    default: return pick_sweep<_Float16, float>(flags, c->esingle, per);
    }
}

// the tiles built for the loaded data fix the block (four waves also with double-precision
// functions, whose registers leave three waves per SIMD)
static int tile_waves(const mpr_ctx* c) { return shape_waves(c->tile_shape); }

static TiledFn tiled_fn(const mpr_ctx* c, int flags)
{
    const bool per = c->cfg.boundary == MPR_PERIODIC;
    const int sh = c->tile_shape;
    switch (c->sprec) {
    case MPR_FP64: return c->fsingle ? pick_tiled<double, float>(flags, per, sh) : pick_tiled<double, double>(flags, per, sh);
    case MPR_FP32: return c->fsingle ? pick_tiled<float, float>(flags, per, sh) : pick_tiled<float, double>(flags, per, sh);
    case MPR_FIX16: return pick_tiled<Fix15, float>(flags, per, sh);
    default: return pick_tiled<_Float16, float>(flags, per, sh);
    }
}

// one sweep of the tiled path: every tile of every (grid, chain), src_buf -> the other buffer
static void enqueue_tiled(mpr_ctx* c, int flags, int sweep_off, int src_buf, const RunCtl* run,
                          uint8_t* dec)
{
    TiledArgs a{};
    a.tiles = c->d_tiles;
    a.gcs = c->d_gcs;
    a.ctl = c->d_ctl;
    a.run = run;
    a.src = c->d_state[src_buf];
    a.dst = c->d_state[1 - src_buf];
    a.acc = c->d_acc;
    a.acc32 = c->d_acc32;
    a.rk_mask = c->d_rk_mask;
    a.rk_base = c->d_rk_base;
    a.dec = dec;
    a.ictl = c->d_ictl;
    a.gacc = c->d_gacc;
    a.econst = c->d_econst;
    a.trace = c->d_trace;
    a.acc_target = c->cfg.acc_target;
    a.T_min = c->cfg.T_min;
    a.T_max = c->cfg.T_max;
    a.q = c->cfg.q;
    a.J = c->cfg.J;
    a.n_gc = (int32_t)c->gcs.size();
    a.n_tiles = c->n_tiles;
    a.sweep_off = sweep_off;
    a.key0 = (uint32_t)(c->cfg.seed & 0xffffffffu);
    a.key1 = (uint32_t)(c->cfg.seed >> 32);
    a.single = c->gcs.size() == 1;
    a.ntx = c->tiles_ntx;
    a.g0 = c->gcs[0];
    a.inv_piq = 1.0 / (3.14159265358979323846 * c->cfg.q);
    const int waves = tile_waves(c);
    hipLaunchKernelGGL(tiled_fn(c, flags), dim3((unsigned)c->n_tiles), dim3(kWave * waves), 0,
                       c->stream, a);
}

static SparseFn sparse_fn(const mpr_ctx* c, int flags, int colour)
{
    const bool per = c->cfg.boundary == MPR_PERIODIC;
    switch (c->sprec) {
    case MPR_FP64: return c->fsingle ? pick_sparse<double, float>(flags, per, colour)
                                     : pick_sparse<double, double>(flags, per, colour);
    case MPR_FP32: return c->fsingle ? pick_sparse<float, float>(flags, per, colour)
                                     : pick_sparse<float, double>(flags, per, colour);
    case MPR_FIX16: return pick_sparse<Fix15, float>(flags, per, colour);
    default: return pick_sparse<_Float16, float>(flags, per, colour);
    }
}

// one sweep of the compacted path: colour 0 then colour 1, in place on the current buffer
static void enqueue_sparse(mpr_ctx* c, int flags, int sweep_off, const RunCtl* run, uint8_t* dec)
{
    for (int col = 0; col < 2; ++col) {
        SparseArgs a{};
        a.sites = c->d_sites;
        a.waves = c->d_waves[col];
        a.lead_wave = c->d_lead[col];
        a.gcs = c->d_gcs;
        a.ctl = c->d_ctl;
        a.run = run;
        a.state = c->d_state[c->cur];
        a.acc = c->d_acc;
        a.acc32 = c->d_acc32;
        a.rk_mask = c->d_rk_mask;
        a.rk_base = c->d_rk_base;
        a.dec = dec;
        a.ictl = c->d_ictl;
        a.gacc = c->d_gacc;
        a.econst = c->d_econst;
        a.trace = c->d_trace;
        a.acc_target = c->cfg.acc_target;
        a.T_min = c->cfg.T_min;
        a.T_max = c->cfg.T_max;
        a.q = c->cfg.q;
        a.J = c->cfg.J;
        a.n_gc = (int32_t)c->gcs.size();
        a.n_waves = c->n_waves[col];
        a.sweep_off = sweep_off;
        a.key0 = (uint32_t)(c->cfg.seed & 0xffffffffu);
        a.key1 = (uint32_t)(c->cfg.seed >> 32);
        a.single = c->gcs.size() == 1;
        a.single_base = c->list_base0[col];
        a.group_waves = c->group_waves;
        a.single_waves = c->list_waves[col];
        const unsigned blocks = (unsigned)((c->n_waves[col] + kWavesPerBlock - 1) / kWavesPerBlock);
        hipLaunchKernelGGL(sparse_fn(c, flags, col), dim3(blocks), dim3(kWave * kWavesPerBlock), 0,
                           c->stream, a);
    }
}

// buffer flips per sweep: the fused path ping-pongs, the compacted path works in place
static inline int flips(const mpr_ctx* c) { return c->sparse ? 0 : 1; }

static void enqueue_sweep(mpr_ctx* c, int flags, int sweep_off, int src_buf, const RunCtl* run,
                          uint8_t* dec)
{
    if (c->sparse) {
        enqueue_sparse(c, flags, sweep_off, run, dec);
        return;
    }
    if (c->tiled) {
        enqueue_tiled(c, flags, sweep_off, src_buf, run, dec);
        return;
    }
    SweepArgs a{};
    a.items = c->d_items;
    a.gcs = c->d_gcs;
    a.ctl = c->d_ctl;
    a.run = run;
    a.src = c->d_state[src_buf];
    a.dst = c->d_state[1 - src_buf];
    a.acc = c->d_acc;
    a.acc32 = c->d_acc32;
    a.rk_mask = c->d_rk_mask;
    a.rk_base = c->d_rk_base;
    a.dec = dec;
    a.e_part = c->d_e_part;
    a.a_part = c->d_a_part;
    a.ictl = c->d_ictl;
    a.gacc = c->d_gacc;
    a.trace = c->d_trace;
    a.acc_target = c->cfg.acc_target;
    a.T_min = c->cfg.T_min;
    a.T_max = c->cfg.T_max;
    a.n_gc = (int32_t)c->gcs.size();
    a.n_items = (int32_t)c->items.size();
    a.sweep_off = sweep_off;
    a.key0 = (uint32_t)(c->cfg.seed & 0xffffffffu);
    a.key1 = (uint32_t)(c->cfg.seed >> 32);
    a.q = c->cfg.q;
    a.J = c->cfg.J;
    a.periodic = c->cfg.boundary == MPR_PERIODIC;
    const unsigned blocks = (unsigned)((c->items.size() + kWavesPerBlock - 1) / kWavesPerBlock);
    SweepFn fn = sweep_fn(c, flags);
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(kWave * kWavesPerBlock), 0, c->stream, a);
}

static void enqueue_control(mpr_ctx* c, int sweep_off)
{
    auto fn = c->esingle ? k_control<true> : k_control<false>;
    hipLaunchKernelGGL(fn, dim3((unsigned)c->gcs.size()), dim3(c->ctl_threads), 0, c->stream, c->d_gcs, c->d_ctl,
                       c->d_run, c->d_e_part, c->d_a_part, c->d_trace, sweep_off, c->cfg.J,
                       c->cfg.acc_target, c->cfg.T_min, c->cfg.T_max);
}

// n sweeps of `mode` starting from buffer c->cur; sweep i reads buffer (cur + i) & 1
static void enqueue_block(mpr_ctx* c, int mode, int n)
{
    const int flags = mode == MODE_EQUIL ? F_ENERGY : (mode == MODE_AVG ? F_ACC : 0);
    int buf = c->cur;
    for (int i = 0; i < n; ++i) {
        enqueue_sweep(c, flags, i, buf, c->d_run, nullptr);
        if (mode == MODE_EQUIL && c->esingle) enqueue_control(c, i);   // else inside the sweeps
        buf ^= flips(c);
    }
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, c->stream, c->d_run, (int64_t)n);
}

// launches the captured graph of `len` sweeps of `mode` from the current buffer (captured at its
// first use and kept until the launch arguments it holds change)
static int launch_graph(mpr_ctx* c, int mode, int len)
{
    const auto key = std::make_tuple(mode, c->cur, len);
    hipGraphExec_t exec = nullptr;
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        enqueue_block(c, mode, len);
        hipGraph_t graph = nullptr;
        HIPCHK(c, hipStreamEndCapture(c->stream, &graph));
        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(c, e);
        c->graphs[key] = exec;
    } else exec = it->second;
    HIPCHK(c, hipGraphLaunch(exec, c->stream));
    return MPR_OK;
}

static int run_sweeps(mpr_ctx* c, int mode, int n)
{
    int done = 0;
    const int K = c->graph_k;
    if (K > 0) {
        // whole graphs of K sweeps (K is even: the buffer parity is unchanged), then one graph of
        // the remaining sweeps
        for (; done + K <= n; done += K) {
            const int rc = launch_graph(c, mode, K);
            if (rc) return rc;
        }
        if (n - done >= 2) {
            const int rc = launch_graph(c, mode, n - done);
            if (rc) return rc;
            if ((n - done) & 1) c->cur ^= flips(c);
            done = n;
        }
    }
    if (done < n) {
        enqueue_block(c, mode, n - done);
        if ((n - done) & 1) c->cur ^= flips(c);
    }
    HIPCHK(c, hipGetLastError());
    c->next_sweep += n;
    return MPR_OK;
}

// n inference sweeps: energy matching from T_0 (fixed = 0), or equilibration at each chain's T
// (kFixT), also with a fixed window (kFixT | kFixAlpha)
static int infer_common(mpr_ctx* c, int32_t n_equil, int fixed, double* T_host)
{
    int rc = MPR_OK;
    const int n_gc = (int)c->gcs.size();
    if (n_equil > c->trace_cap) {
        if (c->d_trace) (void)hipFree(c->d_trace);
        c->d_trace = nullptr;
        HIPCHK(c, hipMalloc(&c->d_trace, (size_t)n_gc * std::max(n_equil, 1) * 4 * sizeof(double)));
        c->trace_cap = n_equil;
        for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);   // captured trace pointer
        c->graphs.clear();
    }
    rc = mark(c, PHASE_INFER, 0);
    if (rc) return rc;
    hipLaunchKernelGGL(k_infer_begin, dim3((3 * n_gc * kAccCopies + 255) / 256), dim3(256), 0, c->stream, c->d_ctl,
                       c->d_ictl, c->d_gacc, (c->sparse || c->tiled) ? c->d_econst : nullptr, n_gc, c->cfg.J,
                       c->cfg.T_min, c->cfg.T_max, c->d_run,
                       (int64_t)(c->next_sweep + n_equil / 2), (int64_t)c->next_sweep,
                       (int64_t)c->trace_cap, (int64_t)n_equil, fixed);
    rc = run_sweeps(c, MODE_EQUIL, n_equil);
    if (rc) return rc;
    hipLaunchKernelGGL(k_infer_end, dim3((n_gc + 255) / 256), dim3(256), 0, c->stream, c->d_gcs,
                       c->d_ctl, c->d_ictl, c->d_gacc, c->d_trace, c->d_run, n_gc, (int)!c->esingle,
                       (int64_t)n_equil, c->cfg.J, c->cfg.acc_target, c->cfg.T_min, c->cfg.T_max);
    HIPCHK(c, hipGetLastError());
    rc = mark(c, PHASE_INFER, 1, n_equil);
    if (rc) return rc;
    c->trace_len = n_equil;
    c->phase = std::max(c->phase, (int)PH_TEMPERED);
    if (T_host) {
        std::vector<GcCtl> ctl(n_gc);
        HIPCHK(c, hipMemcpyAsync(ctl.data(), c->d_ctl, n_gc * sizeof(GcCtl), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int i = 0; i < n_gc; ++i) T_host[i] = ctl[i].T;
    }
    return MPR_OK;
}

int mpr_infer_temperature(mpr_ctx* c, int32_t n_equil, double* T_host)
{
    int rc = usable(c);
    if (rc) return rc;
    if (c->phase < PH_LOADED) return fail(c, MPR_ESTATE, "no data loaded");
    if (n_equil < 0) return fail(c, MPR_EINVAL, "n_equil < 0");
    return infer_common(c, n_equil, 0, T_host);
}

int mpr_equilibrate(mpr_ctx* c, int32_t n, double* T_host)
{
    int rc = usable(c);
    if (rc) return rc;
    if (c->phase < PH_TEMPERED) return fail(c, MPR_ESTATE, "no temperature: infer or set it first");
    if (n < 0) return fail(c, MPR_EINVAL, "n < 0");
    return infer_common(c, n, kFixT, T_host);
}

int mpr_set_temperature_curve(mpr_ctx* c, int32_t n_T, const double* T_host, const double* e_host,
                              double* T_out)
{
    int rc = usable(c);
    if (rc) return rc;
    if (c->phase < PH_LOADED) return fail(c, MPR_ESTATE, "no data loaded");
    if (n_T < 1 || !T_host || !e_host) return fail(c, MPR_EINVAL, "bad curve arguments");
    for (int i = 0; i < n_T; ++i)
        if (!(T_host[i] > 0.0) || !std::isfinite(T_host[i]) || !std::isfinite(e_host[i]) ||
            (i > 0 && !(T_host[i] > T_host[i - 1])))
            return fail(c, MPR_EINVAL, "curve temperatures must be finite, positive and increasing");
    double* d_tab = nullptr;
    HIPCHK(c, hipMalloc(&d_tab, 2 * (size_t)n_T * sizeof(double)));
    hipError_t e1 = h2d(c, d_tab, T_host, n_T * sizeof(double));
    hipError_t e2 = e1 == hipSuccess ? h2d(c, d_tab + n_T, e_host, n_T * sizeof(double)) : e1;
    if (e2 == hipSuccess) {
        const int n_gc = (int)c->gcs.size();
        hipLaunchKernelGGL(k_curve_temperature, dim3((n_gc + 255) / 256), dim3(256), 0, c->stream,
                           c->d_ctl, n_gc, d_tab, d_tab + n_T, n_T);
        e2 = hipGetLastError();
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
    }
    (void)hipFree(d_tab);
    HIPCHK(c, e2);
    c->phase = std::max(c->phase, (int)PH_TEMPERED);
    if (T_out) {
        std::vector<GcCtl> ctl(c->gcs.size());
        HIPCHK(c, hipMemcpyAsync(ctl.data(), c->d_ctl, ctl.size() * sizeof(GcCtl), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < ctl.size(); ++i) T_out[i] = ctl[i].T;
    }
    return MPR_OK;
}

int mpr_set_temperature_curve_noalloc(mpr_ctx* c, int32_t n_T, const double* T_host,
                                      const double* e_host, double* T_out)
{
    int rc = usable(c);
    if (rc) return rc;
    if (c->phase < PH_LOADED) return fail(c, MPR_ESTATE, "no data loaded");
    if (n_T < 1 || !T_host || !e_host) return fail(c, MPR_EINVAL, "bad curve arguments");
    const int n_gc = (int)c->gcs.size();
    if (2 * (int64_t)n_T + (T_out ? n_gc : 0) > kScratchDoubles)
        return fail(c, MPR_EINVAL, "curve of %d points%s exceeds the static scratch of %d doubles",
                    n_T, T_out ? " and the chains' temperatures" : "", kScratchDoubles);
    for (int i = 0; i < n_T; ++i)
        if (!(T_host[i] > 0.0) || !std::isfinite(T_host[i]) || !std::isfinite(e_host[i]) ||
            (i > 0 && !(T_host[i] > T_host[i - 1])))
            return fail(c, MPR_EINVAL, "curve temperatures must be finite, positive and increasing");
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev != c->device) return fail(c, MPR_EINVAL, "the context's device is not the current device");
    double* tab = nullptr;
    HIPCHK(c, scratch_address(dev, &tab));
    // every value the kernels read is written here first: nothing of an earlier call is used
    HIPCHK(c, hipMemcpyAsync(tab, T_host, n_T * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(tab + n_T, e_host, n_T * sizeof(double), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_curve_temperature, dim3((n_gc + 255) / 256), dim3(256), 0, c->stream,
                       c->d_ctl, n_gc, tab, tab + n_T, n_T);
    if (T_out)
        hipLaunchKernelGGL(k_gather_T, dim3((n_gc + 255) / 256), dim3(256), 0, c->stream, c->d_ctl,
                           n_gc, tab + 2 * n_T);
    HIPCHK(c, hipGetLastError());
    if (T_out)
        HIPCHK(c, hipMemcpyAsync(T_out, tab + 2 * n_T, n_gc * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
    // the host arrays may be released, and another call may reuse the scratch, after this
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->phase = std::max(c->phase, (int)PH_TEMPERED);
    return MPR_OK;
}

int mpr_energy_curve(const mpr_config* cfg, void* hip_stream, int32_t side, int32_t n_T,
                     const double* T_host, int32_t n_burn, int32_t n_meas, double* e_host,
                     double* trace_host)
{
    if (!cfg || !T_host || !e_host || n_T < 1 || n_burn < 0 || n_meas < 1) return MPR_EINVAL;
    if (n_burn > INT32_MAX - n_meas) return MPR_EINVAL;
    for (int i = 0; i < n_T; ++i)
        if (!(T_host[i] > 0.0) || !std::isfinite(T_host[i])) return MPR_EINVAL;
    mpr_config k = *cfg;
    k.boundary = MPR_PERIODIC;
    k.n_chains = n_T;
    k.sweep_mode = MPR_SWEEP_FUSED;
    if (k.tile_rows < 0) k.tile_rows = 0;
    mpr_ctx* c = nullptr;
    int rc = mpr_create(&k, hip_stream, &c);
    if (rc) return rc;
    const int64_t H = side, W = side;
    rc = setup_shapes(c, 1, &H, &W);
    // no data: a zero field and an all-zero mask, every site free
    double* d_z = nullptr;
    uint8_t* d_m = nullptr;
    if (!rc && (hipMalloc(&d_z, (size_t)H * W * sizeof(double)) != hipSuccess ||
                hipMalloc(&d_m, (size_t)H * W) != hipSuccess ||
                hipMemsetAsync(d_z, 0, (size_t)H * W * sizeof(double), c->stream) != hipSuccess ||
                hipMemsetAsync(d_m, 0, (size_t)H * W, c->stream) != hipSuccess))
        rc = MPR_ENOMEM;
    if (!rc) rc = load_common(c, d_z, d_m, true);
    if (!rc) {
        std::vector<GcCtl> ctl(n_T);
        if (hipMemcpyAsync(ctl.data(), c->d_ctl, n_T * sizeof(GcCtl), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            rc = MPR_EHIP;
        for (int i = 0; i < n_T && !rc; ++i) ctl[i].T = T_host[i];
        if (!rc && h2d(c, c->d_ctl, ctl.data(), n_T * sizeof(GcCtl)) != hipSuccess) rc = MPR_EHIP;
    }
    // burn-in with the window control, then measurement sweeps with the window fixed
    const int32_t total = n_burn + n_meas;
    std::vector<double> tr((size_t)std::max(n_burn, n_meas) * 4);
    for (int part = 0; part < 2 && !rc; ++part) {
        const int32_t n = part ? n_meas : n_burn;
        if (n == 0) continue;
        c->phase = PH_TEMPERED;
        rc = infer_common(c, n, part ? kFixT | kFixAlpha : kFixT, nullptr);
        for (int i = 0; i < n_T && !rc; ++i) {
            int32_t got = 0;
            rc = mpr_get_trace(c, i, n, tr.data(), &got);
            if (!rc && got != n) rc = MPR_EHIP;
            if (rc) break;
            if (trace_host)
                std::memcpy(trace_host + ((size_t)i * total + (part ? n_burn : 0)) * 4, tr.data(),
                            (size_t)n * 4 * sizeof(double));
            if (part) {
                double s = 0.0;
                for (int32_t t = 0; t < n; ++t) s += tr[(size_t)t * 4];
                e_host[i] = s / (double)n;
            }
        }
    }
    mpr_destroy(c);
    if (d_z) (void)hipFree(d_z);
    if (d_m) (void)hipFree(d_m);
    return rc;
}

int mpr_set_temperature(mpr_ctx* c, double T)
{
    int rc = usable(c);
    if (rc) return rc;
    if (c->phase < PH_LOADED) return fail(c, MPR_ESTATE, "no data loaded");
    if (!(T > 0.0) || !std::isfinite(T)) return fail(c, MPR_EINVAL, "temperature must be > 0");
    std::vector<GcCtl> ctl(c->gcs.size());
    HIPCHK(c, hipMemcpyAsync(ctl.data(), c->d_ctl, ctl.size() * sizeof(GcCtl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto& k : ctl) k.T = T;
    HIPCHK(c, hipMemcpyAsync(c->d_ctl, ctl.data(), ctl.size() * sizeof(GcCtl), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->phase = std::max(c->phase, (int)PH_TEMPERED);
    return MPR_OK;
}

int mpr_burn_in(mpr_ctx* c, int32_t n)
{
    int rc = usable(c);
    if (rc) return rc;
    if (n < 0) return fail(c, MPR_EINVAL, "n < 0");
    if (c->phase < PH_TEMPERED) return fail(c, MPR_ESTATE, "no temperature: infer or set it first");
    return run_sweeps(c, MODE_BURN, n);
}

// acc[i] += acc32[i] 2^-24, acc32[i] = 0: exact (both are whole multiples of 2^-24 far below
// 2^29), so the FP64 sums equal those of adding each sweep's FP16 value in double precision
__global__ __launch_bounds__(256) void k_acc_fold(double* acc, uint32_t* acc32, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = acc32[i];
        acc[i] += (double)v * 0x1p-24;
        acc32[i] = 0u;
    }
}

// FP16 averaging sweeps sum into 32-bit words (kAcc32): at most 2^24 units per sweep (a value
// of 1), so 128 sweeps stay below 2^31
constexpr int kAcc32Sweeps = 128;

int mpr_run(mpr_ctx* c, int32_t n_avg)
{
    int rc = usable(c);
    if (rc) return rc;
    if (n_avg < 0) return fail(c, MPR_EINVAL, "n_avg < 0");
    if (c->phase < PH_TEMPERED) return fail(c, MPR_ESTATE, "no temperature: infer or set it first");
    rc = mark(c, PHASE_RUN, 0);
    if (c->d_acc32) {
        const unsigned blocks = (unsigned)std::min<int64_t>(4096, (c->chain_sites + 255) / 256);
        for (int64_t done = 0; !rc && done < n_avg; done += kAcc32Sweeps) {
            rc = run_sweeps(c, MODE_AVG, (int)std::min<int64_t>(kAcc32Sweeps, n_avg - done));
            if (rc) return rc;
            hipLaunchKernelGGL(k_acc_fold, dim3(std::max(blocks, 1u)), dim3(256), 0, c->stream, c->d_acc, c->d_acc32,
                               c->chain_sites);
            HIPCHK(c, hipGetLastError());
        }
    } else if (!rc) {
        rc = run_sweeps(c, MODE_AVG, n_avg);
    }
    if (!rc) rc = mark(c, PHASE_RUN, 1, n_avg);
    if (rc) return rc;
    c->n_avg += n_avg;
    if (n_avg > 0) c->phase = PH_AVERAGED;
    return MPR_OK;
}

int mpr_get_predictions(mpr_ctx* c, double* zhat)
{
    int rc = usable(c);
    if (rc) return rc;
    if (!zhat) return fail(c, MPR_EINVAL, "null output");
    if (c->phase < PH_AVERAGED || c->n_avg == 0) return fail(c, MPR_ESTATE, "no averaging sweep yet");
    int64_t max_sites = 0;
    for (int g = 0; g < c->G; ++g) max_sites = std::max(max_sites, c->H[g] * c->W[g]);
    const dim3 grid = site_grid(max_sites, c->G);
    rc = mark(c, PHASE_PREDICT, 0);
    if (rc) return rc;
    switch (c->sprec) {
    case MPR_FP64: hipLaunchKernelGGL(k_finalize<double>, grid, dim3(256), 0, c->stream, c->d_gcs, c->d_gi, c->d_state[c->cur], c->d_acc, c->d_rk_mask, c->d_rk_base, c->d_zcopy, zhat, c->C, c->n_avg); break;
    case MPR_FP32: hipLaunchKernelGGL(k_finalize<float>, grid, dim3(256), 0, c->stream, c->d_gcs, c->d_gi, c->d_state[c->cur], c->d_acc, c->d_rk_mask, c->d_rk_base, c->d_zcopy, zhat, c->C, c->n_avg); break;
    case MPR_FIX16: hipLaunchKernelGGL(k_finalize<Fix15>, grid, dim3(256), 0, c->stream, c->d_gcs, c->d_gi, c->d_state[c->cur], c->d_acc, c->d_rk_mask, c->d_rk_base, c->d_zcopy, zhat, c->C, c->n_avg); break;
    default: hipLaunchKernelGGL(k_finalize<_Float16>, grid, dim3(256), 0, c->stream, c->d_gcs, c->d_gi, c->d_state[c->cur], c->d_acc, c->d_rk_mask, c->d_rk_base, c->d_zcopy, zhat, c->C, c->n_avg); break;
    }
    HIPCHK(c, hipGetLastError());
    return mark(c, PHASE_PREDICT, 1);
}

int mpr_get_timings(mpr_ctx* c, mpr_timings* out)
{
    if (!c || !out) return MPR_EINVAL;
    double* ms[4] = {&out->load_ms, &out->infer_ms, &out->run_ms, &out->predict_ms};
    for (int p = 0; p < 4; ++p) {
        *ms[p] = -1.0;
        if (!c->ev_done[p]) continue;
        HIPCHK(c, hipEventSynchronize(c->ev[p][1]));
        float t = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&t, c->ev[p][0], c->ev[p][1]));
        *ms[p] = t;
    }
    out->infer_sweeps = c->ev_done[PHASE_INFER] ? c->ev_sweeps[PHASE_INFER] : 0;
    out->run_sweeps = c->ev_done[PHASE_RUN] ? c->ev_sweeps[PHASE_RUN] : 0;
    return MPR_OK;
}

int mpr_get_stats(mpr_ctx* c, mpr_chain_stats* out)
{
    int rc = usable(c);
    if (rc) return rc;
    if (!out) return fail(c, MPR_EINVAL, "null output");
    if (c->phase < PH_LOADED) return fail(c, MPR_ESTATE, "no data loaded");
    std::vector<GcCtl> ctl(c->gcs.size());
    HIPCHK(c, hipMemcpyAsync(ctl.data(), c->d_ctl, ctl.size() * sizeof(GcCtl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < ctl.size(); ++i) {
        const GcDesc& d = c->gcs[i];
        const GridInfo& G = c->gi[d.grid];
        mpr_chain_stats& s = out[i];
        s.T = ctl[i].T; s.alpha = ctl[i].alpha; s.e_sample = ctl[i].e_smp; s.e_sim = ctl[i].e_sim;
        s.acc_rate = ctl[i].acc_rate; s.n_pred = d.n_pred; s.n_bonds = d.n_bonds;
        s.n_sample_bonds = G.n_sample_bonds; s.zmin = G.zmin; s.zmax = G.zmax;
    }
    return MPR_OK;
}

int mpr_get_trace(mpr_ctx* c, int32_t gc, int32_t max_entries, double* out, int32_t* n_out)
{
    int rc = usable(c);
    if (rc) return rc;
    if (!out || gc < 0 || gc >= (int)c->gcs.size() || max_entries < 0)
        return fail(c, MPR_EINVAL, "bad trace request");
    const int64_t n = std::min<int64_t>(c->trace_len, max_entries);
    if (n > 0) {
        HIPCHK(c, hipMemcpyAsync(out, c->d_trace + (size_t)gc * c->trace_cap * 4, n * 4 * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (n_out) *n_out = (int32_t)n;
    return MPR_OK;
}

static dim3 gc_grid(const mpr_ctx* c)
{
    int64_t m = 0;
    for (int g = 0; g < c->G; ++g) m = std::max(m, c->H[g] * c->W[g]);
    return site_grid(m, (int)c->gcs.size());
}

int mpr_get_state(mpr_ctx* c, double* u, double* acc, double* ctl_host, int64_t* meta)
{
    int rc = usable(c);
    if (rc) return rc;
    if (c->phase < PH_LOADED) return fail(c, MPR_ESTATE, "no data loaded");
    if (u || acc) {
        switch (c->sprec) {
        case MPR_FP64: launch_get_state<double>(c, u, acc, gc_grid(c)); break;
        case MPR_FP32: launch_get_state<float>(c, u, acc, gc_grid(c)); break;
        case MPR_FIX16: launch_get_state<Fix15>(c, u, acc, gc_grid(c)); break;
        default: launch_get_state<_Float16>(c, u, acc, gc_grid(c)); break;
        }
        HIPCHK(c, hipGetLastError());
    }
    if (ctl_host) {
        std::vector<GcCtl> ctl(c->gcs.size());
        HIPCHK(c, hipMemcpyAsync(ctl.data(), c->d_ctl, ctl.size() * sizeof(GcCtl), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < ctl.size(); ++i) { ctl_host[2 * i] = ctl[i].T; ctl_host[2 * i + 1] = ctl[i].alpha; }
    }
    if (meta) { meta[0] = c->next_sweep; meta[1] = c->n_avg; meta[2] = c->phase; }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MPR_OK;
}

int mpr_set_state(mpr_ctx* c, const double* u, const double* acc, const double* ctl_host,
                  const int64_t* meta)
{
    int rc = usable(c);
    if (rc) return rc;
    if (c->phase < PH_LOADED) return fail(c, MPR_ESTATE, "no data loaded");
    if (meta && (meta[0] < 0 || meta[1] < 0 || meta[2] < PH_LOADED || meta[2] > PH_AVERAGED))
        return fail(c, MPR_EINVAL, "bad checkpoint metadata");
    if (ctl_host)
        for (size_t i = 0; i < c->gcs.size(); ++i)
            if (!(ctl_host[2 * i] > 0.0) || !(ctl_host[2 * i + 1] > 0.0 && ctl_host[2 * i + 1] <= 1.0))
                return fail(c, MPR_EINVAL, "bad temperature or window in checkpoint");
    if (u) {
        HIPCHK(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
        switch (c->sprec) {
        case MPR_FP64: launch_set_state<double>(c, u, nullptr, 0, gc_grid(c)); break;
        case MPR_FP32: launch_set_state<float>(c, u, nullptr, 0, gc_grid(c)); break;
        case MPR_FIX16: launch_set_state<Fix15>(c, u, nullptr, 0, gc_grid(c)); break;
        default: launch_set_state<_Float16>(c, u, nullptr, 0, gc_grid(c)); break;
        }
        int flag = 0;
        HIPCHK(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (flag) return fail(c, MPR_EINVAL, "checkpoint angle outside [0, 1] at a prediction site");
    }
    if (u || acc) {
        switch (c->sprec) {
        case MPR_FP64: launch_set_state<double>(c, u, acc, 1, gc_grid(c)); break;
        case MPR_FP32: launch_set_state<float>(c, u, acc, 1, gc_grid(c)); break;
        case MPR_FIX16: launch_set_state<Fix15>(c, u, acc, 1, gc_grid(c)); break;
        default: launch_set_state<_Float16>(c, u, acc, 1, gc_grid(c)); break;
        }
        HIPCHK(c, hipGetLastError());
    }
    if (ctl_host) {
        std::vector<GcCtl> ctl(c->gcs.size());
        HIPCHK(c, hipMemcpyAsync(ctl.data(), c->d_ctl, ctl.size() * sizeof(GcCtl), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < ctl.size(); ++i) { ctl[i].T = ctl_host[2 * i]; ctl[i].alpha = ctl_host[2 * i + 1]; }
        HIPCHK(c, hipMemcpyAsync(c->d_ctl, ctl.data(), ctl.size() * sizeof(GcCtl), hipMemcpyHostToDevice, c->stream));
    }
    if (meta) {
        c->next_sweep = meta[0];
        c->n_avg = meta[1];
        c->phase = (int)meta[2];
        hipLaunchKernelGGL(k_set_base, dim3(1), dim3(1), 0, c->stream, c->d_run, (int64_t)c->next_sweep);
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MPR_OK;
}

int mpr_debug_sweep(mpr_ctx* c, int32_t sweep, uint8_t* dec)
{
    int rc = usable(c);
    if (rc) return rc;
    if (!dec || sweep < 0) return fail(c, MPR_EINVAL, "bad debug sweep arguments");
    if (c->phase < PH_TEMPERED) return fail(c, MPR_ESTATE, "no temperature: infer or set it first");
    int64_t total = 0;
    for (int g = 0; g < c->G; ++g) total += c->H[g] * c->W[g] * c->C;
    HIPCHK(c, hipMemsetAsync(dec, 0, (size_t)total, c->stream));
    hipLaunchKernelGGL(k_set_base, dim3(1), dim3(1), 0, c->stream, c->d_dbg_run, (int64_t)sweep);
    enqueue_sweep(c, F_DEC, 0, c->cur, c->d_dbg_run, dec);
    c->cur ^= flips(c);
    HIPCHK(c, hipGetLastError());
    return MPR_OK;
}

int mpr_bench_sweeps(mpr_ctx* c, int32_t n)
{
    int rc = usable(c);
    if (rc) return rc;
    if (n < 0) return fail(c, MPR_EINVAL, "n < 0");
    if (c->phase < PH_TEMPERED) return fail(c, MPR_ESTATE, "no temperature: infer or set it first");
    int buf = c->cur;
    for (int i = 0; i < n; ++i) {
        enqueue_sweep(c, F_ENERGY, i, buf, c->d_run, nullptr);
        buf ^= flips(c);
    }
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, c->stream, c->d_run, (int64_t)n);
    c->cur = buf;
    c->next_sweep += n;
    HIPCHK(c, hipGetLastError());
    return MPR_OK;
}

// ------------------------------------------------------------------ autotuning
// Rows per work item trade parallelism (more, shorter items) against the 4 halo rows each item
// recomputes.  The sweep's results do not depend on the choice (tested bitwise), so the tuner
// may pick any candidate; it times n inference sweeps per candidate from a saved state, restores
// the state, and remembers the winner per shape signature (in memory, and in the text file named
// by MPR_TUNE_CACHE if set).  The table is shared by every context of the process: callers hold
// tune_mutex() while they use it.
static std::mutex& tune_mutex()
{
    static std::mutex m;
    return m;
}
// A tuned choice: sweep path, rows per work item of the fused path, block shape of the tiled path
// (-1: the automatic rule) and sweeps per captured graph (0: the configured value).
struct TuneChoice { int path, rows, shape, graph_k; };

static std::map<std::string, TuneChoice>& tune_cache()
{
    static std::map<std::string, TuneChoice> m;
    static bool loaded = false;
    if (!loaded) {
        loaded = true;
        if (const char* path = std::getenv("MPR_TUNE_CACHE")) {
            if (FILE* f = std::fopen(path, "r")) {
                char key[256];
                TuneChoice t;
                while (std::fscanf(f, "%255s %d %d %d %d", key, &t.path, &t.rows, &t.shape, &t.graph_k) == 5)
                    m[key] = t;
                std::fclose(f);
            }
        }
    }
    return m;
}

static std::string tune_key(const mpr_ctx* c)
{
    uint64_t h = 1469598103934665603ull;
    int64_t P = 0, N = 0;
    for (int g = 0; g < c->G; ++g) {
        for (int64_t v : {c->H[g], c->W[g]}) { h ^= (uint64_t)v; h *= 1099511628211ull; }
        P += c->gi[g].n_pred;
        N += c->H[g] * c->W[g];
    }
    // the path depends on the share of prediction sites: keyed to the percent
    const int pct = N > 0 ? (int)std::lround(100.0 * (double)P / (double)N) : 0;
    char buf[192];
    std::snprintf(buf, sizeof buf, "s%d_f%d_e%d_b%d_c%d_g%d_m%d_t%d_k%d_p%d_%016llx", c->sprec, (int)c->fsingle,
                  (int)c->esingle, c->cfg.boundary, c->C, c->G, c->cfg.sweep_mode, c->cfg.tile_shape,
                  c->cfg.graph_sweeps, pct, (unsigned long long)h);
    return buf;
}

static int use_rows(mpr_ctx* c, int rows)
{
    c->rows = rows;
    build_items(c, rows);
    if ((int64_t)c->items.size() > c->item_cap) return fail(c, MPR_EINVAL, "too many work items");
    HIPCHK(c, h2d(c, c->d_items, c->items.data(), c->items.size() * sizeof(Item)));
    HIPCHK(c, h2d(c, c->d_gcs, c->gcs.data(), c->gcs.size() * sizeof(GcDesc)));
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    c->alloc_sig.clear();     // buffers stay, but a reload must rebuild the signature
    return MPR_OK;
}

// the tile shape the automatic rule gives this context (see build_tiles_t)
static int rule_shape(const mpr_ctx* c)
{
    if (!c->fsingle) return kShapeW4Base;
    const int base_rows = (c->sprec == MPR_FP64) ? 8 : 16;   // tile_rows<S, float>()
    int64_t base = 0;
    for (const GcDesc& d : c->gcs)
        base += (int64_t)((d.H + base_rows - 1) / base_rows) * ((d.wc + kTileCols - 1) / kTileCols);
    return base < kTileWavesSwitch ? kShapeW8Tall : kShapeW4Base;
}

static const int kGraphCandidates[] = {16, 32, 64};
static bool tune_graphs(const mpr_ctx* c) { return c->cfg.graph_sweeps == 0 && c->stream != nullptr; }

// whether a remembered choice can be used by this context
static bool choice_valid(const mpr_ctx* c, const TuneChoice& t, bool pick_path)
{
    const bool path_ok = t.path == MPR_SWEEP_FUSED || (t.path == MPR_SWEEP_SPARSE && sparse_possible(c)) ||
                         (t.path == MPR_SWEEP_TILED && tiled_possible(c));
    const bool rows_ok = std::find(std::begin(kRowCandidates), std::end(kRowCandidates), t.rows) !=
                         std::end(kRowCandidates);
    const bool shape_ok = t.shape == -1 || (t.shape >= 0 && t.shape < kTileShapes && (c->fsingle || t.shape == kShapeW4Base));
    const bool graph_ok = t.graph_k == 0 || std::find(std::begin(kGraphCandidates), std::end(kGraphCandidates),
                                                       t.graph_k) != std::end(kGraphCandidates);
    return path_ok && rows_ok && shape_ok && graph_ok && (pick_path || t.path == current_path(c));
}

// Times n inference-variant sweeps of each candidate from the current state (restored after
// each) and keeps the fastest: the row count of the fused path's work items; with sweep_mode AUTO
// the sweep path itself (fused, compacted, tiled); on the tiled path, unless the configuration
// forces one, its block shape (waves per block and tile height); and, when graph_sweeps is 0,
// the sweeps per captured graph (timed as graph replays).  Results do not depend on the row
// count, the tile shape or the graph length (tested bitwise); the path changes only the
// rounding of the energy sums.  Winners are cached per shape, configuration and share of
// prediction sites.
static int autotune(mpr_ctx* c, int n, int* best_out)
{
    const bool pick_path = c->cfg.sweep_mode == MPR_SWEEP_AUTO;
    const bool pick_shape = c->cfg.tile_shape == 0;
    const std::string key = tune_key(c);
    auto finish = [&](const TuneChoice& t) -> int {
        int rc = MPR_OK;
        const bool was_tiled = c->tiled;
        const int old_shape = c->tile_shape;
        if (t.rows != c->rows) rc = use_rows(c, t.rows);        // drops the graphs itself
        if (!rc && pick_shape) c->tile_shape_req = t.path == MPR_SWEEP_TILED ? t.shape : -1;
        if (!rc) rc = apply_path(c, t.path);                     // drops them on a path change
        if (!rc && was_tiled && c->tiled && c->tile_shape != old_shape) {
            // another tile shape changes the launches the graphs hold
            for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
            c->graphs.clear();
        }
        // graphs are kept per length: another length needs no drop
        if (!rc && t.graph_k > 0 && tune_graphs(c)) c->graph_k = t.graph_k;
        if (best_out) *best_out = c->rows;
        return rc;
    };
    {
        TuneChoice t{};
        bool hit = false;
        {
            std::lock_guard<std::mutex> lock(tune_mutex());
            auto& cache = tune_cache();
            auto it = cache.find(key);
            if (it != cache.end()) { t = it->second; hit = true; }
        }
        // a remembered winner (possibly read from a file) is used only if this context can use
        // it; otherwise the tuner times again
        if (hit && choice_valid(c, t, pick_path)) return finish(t);
    }
    if (!pick_path && c->sparse) {       // nothing to tune on the compacted path but the graphs
        if (best_out) *best_out = c->rows;
        if (!tune_graphs(c)) return MPR_OK;
    }

    int maxH = 0;
    for (int g = 0; g < c->G; ++g) maxH = std::max<int>(maxH, (int)c->H[g]);
    void* saved = nullptr;
    HIPCHK(c, hipMalloc(&saved, c->plane_elems * c->elem));
    HIPCHK(c, hipMemcpyAsync(saved, c->d_state[c->cur], c->plane_elems * c->elem, hipMemcpyDeviceToDevice, c->stream));
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    auto restore = [&]() -> int {
        HIPCHK(c, hipMemcpyAsync(c->d_state[c->cur], saved, c->plane_elems * c->elem, hipMemcpyDeviceToDevice, c->stream));
        return MPR_OK;
    };
    // one candidate: n sweeps after a warm-up one, then the saved state back
    auto time_sweeps = [&](float& ms) -> int {
        int buf = c->cur;
        enqueue_sweep(c, F_ENERGY, 0, buf, c->d_run, nullptr);
        buf ^= flips(c);
        HIPCHK(c, hipEventRecord(e0, c->stream));
        for (int i = 0; i < n; ++i) { enqueue_sweep(c, F_ENERGY, 0, buf, c->d_run, nullptr); buf ^= flips(c); }
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        return restore();
    };
    // one graph length: a graph of K sweeps captured and replayed until about 4 n sweeps ran;
    // time per sweep
    auto time_graph = [&](int K, float& ms_per_sweep) -> int {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        int buf = c->cur;
        for (int i = 0; i < K; ++i) { enqueue_sweep(c, F_ENERGY, i, buf, c->d_run, nullptr); buf ^= flips(c); }
        HIPCHK(c, hipStreamEndCapture(c->stream, &graph));
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(c, ei);
        const int reps = std::max(1, (4 * n + K - 1) / K);
        hipError_t e = hipGraphLaunch(exec, c->stream);                      // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(exec, c->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        (void)hipGraphExecDestroy(exec);
        HIPCHK(c, e);
        ms_per_sweep = ms / (float)(reps * K);
        return restore();
    };
    // the other paths keep the rows per work item the context had (they do not use them)
    const int rows0 = c->rows;
    TuneChoice best{current_path(c), rows0, c->tile_shape_req, 0};
    int rc = MPR_OK;
    // the candidates: the fused path's row counts (the six best of the cost model and the rule's
    // count), the compacted path, the tiled path's block shapes (one with double-precision
    // functions, or the forced one)
    std::vector<TuneChoice> cands;
    if (pick_path || best.path == MPR_SWEEP_FUSED) {
        std::vector<std::pair<double, int>> ranked;
        for (int r : kRowCandidates) {
            if (r > maxH && r > 2) break;
            ranked.push_back({rows_cost(c, r), r});
        }
        std::sort(ranked.begin(), ranked.end());
        if (ranked.size() > 6) ranked.resize(6);
        const int rule = choose_rows(c);
        if (std::none_of(ranked.begin(), ranked.end(), [&](const std::pair<double, int>& x) { return x.second == rule; }))
            ranked.push_back({0.0, rule});
        for (const auto& x : ranked) cands.push_back({MPR_SWEEP_FUSED, x.second, -1, 0});
    }
    if ((pick_path || best.path == MPR_SWEEP_SPARSE) && sparse_possible(c))
        cands.push_back({MPR_SWEEP_SPARSE, rows0, -1, 0});
    if ((pick_path || best.path == MPR_SWEEP_TILED) && tiled_possible(c)) {
        std::vector<int> shapes;
        if (!pick_shape) shapes.push_back(c->cfg.tile_shape - 1);
        else if (!c->fsingle) shapes.push_back(kShapeW4Base);
        else shapes = {kShapeW4Base, kShapeW8Tall, kShapeW4Tall, kShapeW8Base};
        for (int sh : shapes) cands.push_back({MPR_SWEEP_TILED, rows0, sh, 0});
    }
    // three interleaved rounds over the candidates, the fastest time of each counts (a first
    // candidate timed while the clocks still ramp up would otherwise lose); large workloads time
    // three times the sweeps (differences between candidates are a few per cent there)
    int64_t work = 0;
    for (int g = 0; g < c->G; ++g) work += c->H[g] * c->W[g] * c->C;
    if (work > ((int64_t)1 << 24)) n *= 3;
    std::vector<float> best_t(cands.size(), 1e30f);
    for (int round = 0; round < 3 && !rc; ++round)
        for (size_t k = 0; k < cands.size() && !rc; ++k) {
            const TuneChoice& t = cands[k];
            float ms = 0.0f;
            if (t.path == MPR_SWEEP_FUSED && t.rows != c->rows) rc = use_rows(c, t.rows);
            if (!rc && t.path == MPR_SWEEP_TILED) {
                c->tile_shape_req = t.shape;
                for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
                c->graphs.clear();
            }
            if (!rc) rc = apply_path(c, t.path);
            if (!rc) rc = time_sweeps(ms);
            if (!rc) best_t[k] = std::min(best_t[k], ms);
        }
    c->tile_shape_req = pick_shape ? -1 : c->cfg.tile_shape - 1;
    float best_ms = 1e30f;
    for (size_t k = 0; k < cands.size(); ++k)
        if (best_t[k] < best_ms) {
            best_ms = best_t[k];
            best = cands[k];
            if (best.path == MPR_SWEEP_TILED && !pick_shape) best.shape = -1;
        }
    // the rule's own configuration stays unless a candidate beats it by more than 3 % (timings
    // of candidates a few per cent apart vary between runs)
    {
        const int rule_path = pick_path ? auto_path(c) : current_path(c);
        const int rule_rows = choose_rows(c);
        for (size_t k = 0; k < cands.size(); ++k) {
            const TuneChoice& t = cands[k];
            const bool is_rule = t.path == rule_path &&
                                 (t.path != MPR_SWEEP_FUSED || t.rows == rule_rows) &&
                                 (t.path != MPR_SWEEP_TILED || t.shape == rule_shape(c));
            if (is_rule && best_t[k] <= 1.03f * best_ms) {
                best = t;
                if (best.path == MPR_SWEEP_TILED) best.shape = -1;
                break;
            }
        }
    }
    // sweeps per graph, on the winning path
    if (!rc && tune_graphs(c)) {
        rc = finish(best);
        float best_g[3] = {1e30f, 1e30f, 1e30f};
        for (int round = 0; round < 2 && !rc; ++round)
            for (int i = 0; i < 3 && !rc; ++i) {
                float ms = 0.0f;
                rc = time_graph(kGraphCandidates[i], ms);
                if (!rc) best_g[i] = std::min(best_g[i], ms);
            }
        float bg = 1e30f;
        for (int i = 0; i < 3; ++i)
            if (best_g[i] < bg) { bg = best_g[i]; best.graph_k = kGraphCandidates[i]; }
        if (best_g[1] <= 1.03f * bg) best.graph_k = kGraphCandidates[1];   // the default, 32, unless clearly slower
    }
    (void)hipStreamSynchronize(c->stream);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(saved);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lock(tune_mutex());
        auto& cache = tune_cache();
        cache[key] = best;
        if (const char* path = std::getenv("MPR_TUNE_CACHE")) {
            if (FILE* f = std::fopen(path, "a")) {
                std::fprintf(f, "%s %d %d %d %d\n", key.c_str(), best.path, best.rows, best.shape, best.graph_k);
                std::fclose(f);
            }
        }
    }
    return finish(best);
}

int mpr_autotune(mpr_ctx* c, int32_t n_sweeps, int32_t* rows_out)
{
    int rc = usable(c);
    if (rc) return rc;
    if (c->phase < PH_LOADED) return fail(c, MPR_ESTATE, "no data loaded");
    if (n_sweeps < 1) return fail(c, MPR_EINVAL, "n_sweeps must be >= 1");
    int best = 0;
    rc = autotune(c, n_sweeps, &best);
    if (rows_out) *rows_out = best;
    return rc;
}

int mpr_get_tuning(mpr_ctx* c, int32_t* path, int32_t* rows, int32_t* tile_shape, int32_t* graph_sweeps)
{
    if (!c) return MPR_EINVAL;
    if (c->phase < PH_LOADED) return fail(c, MPR_ESTATE, "no data loaded");
    if (path) *path = current_path(c);
    if (rows) *rows = c->rows;
    if (tile_shape) *tile_shape = c->tiled ? c->tile_shape : -1;
    if (graph_sweeps) *graph_sweeps = c->graph_k;
    return MPR_OK;
}

int mpr_get_sweep_mode(mpr_ctx* c, int32_t* mode_out)
{
    if (!c || !mode_out) return MPR_EINVAL;
    if (c->phase < PH_LOADED) return fail(c, MPR_ESTATE, "no data loaded");
    *mode_out = current_path(c);
    return MPR_OK;
}

int mpr_get_shape(mpr_ctx* c, int32_t* n_grids, int32_t* n_chains, int64_t* n_sites)
{
    if (!c) return MPR_EINVAL;
    if (n_grids) *n_grids = c->G;
    if (n_chains) *n_chains = c->C;
    if (n_sites) *n_sites = c->n_grid_sites;
    return MPR_OK;
}

}  // extern "C"
