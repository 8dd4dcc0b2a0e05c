// swim_pairsum.h -- device building blocks shared by the persistent forward
// kernels (filament and full sperm model): the dense regularized-Brinkmanlet
// pair sum of eq. (BrV) in the symmetric lane schedule, the FP32 kernel
// table's LDS copy, and the compensated (hi, lo) position update.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "swim_math.h"

namespace swim {

template <typename T> struct alignas(4 * sizeof(T)) Src4 {
    T x, y, fx, fy;
};

template <typename T> struct alignas(2 * sizeof(T)) V2 {
    T x, y;
};

// position outside the run bound |x| <= 1e3 (or not finite)
__device__ __forceinline__ bool bad_t(float x) { return !(fabsf(x) <= 1e3f); }
__device__ __forceinline__ bool bad_t(double x) { return !(fabs(x) <= 1e3); }

// copy one system's FP32 kernel table from HBM into LDS (nthreads threads)
__device__ __forceinline__ void tab_load(const TabSys* g, TabSys* tab, int tid, int nthreads)
{
    const float4* src = reinterpret_cast<const float4*>(g);
    float4* dst = reinterpret_cast<float4*>(tab);
    constexpr int NV = (int)(sizeof(TabSys) / sizeof(float4));
    for (int i = tid; i < NV; i += nthreads) dst[i] = src[i];
}

// The FP32 table as a 64 KiB index window: the entry of index id (the bits
// of v >> TAB_SHIFT, TAB_BIAS for v = 1) sits at byte (id << 5) mod 2^16,
// so the address of a pair's entry is (bits >> (TAB_SHIFT - 5)) & 0xFFE0:
// two operations, no bias and no clamp.  Entries 16.. of the table fill
// bytes [0, 32 (TAB_N - 16)), entries 0..15 (v in [1, 2)) the top 512
// bytes, and every other slot is zero: the indices of finite v beyond the
// table (TAB_END .. 4079) land on zeros, as the zero entry TAB_N does for a
// clamped index.  Non-finite v (4080..4095) alias entries 0..15; their
// positions are non-finite already and end the run.
constexpr uint32_t TAB_WIN_BYTES = 65536;
static_assert(TAB_M == 4 && sizeof(TabE) == 32 && TAB_BIAS == 2032 && TAB_END <= 4080,
              "the index window holds 2048 entries of v's octaves 0..127");
__device__ __forceinline__ uint32_t tab_win_off(uint32_t bits) { return (bits >> (TAB_SHIFT - 5)) & 0xFFE0u; }

// copy one system's FP32 kernel table from HBM into its LDS index window
__device__ __forceinline__ void tab_load_window(const TabSys* g, unsigned char* win, int tid, int nthreads)
{
    const float4* src = reinterpret_cast<const float4*>(g->e);
    float4* dst = reinterpret_cast<float4*>(win);
    constexpr int NV = (int)(TAB_WIN_BYTES / sizeof(float4)), EV = (int)(sizeof(TabE) / sizeof(float4));
    for (int i = tid; i < NV; i += nthreads) {
        // slot id mod 2048 holds entry id - TAB_BIAS
        const int ent = (i / EV - (int)TAB_BIAS) & 2047;
        dst[i] = ent < TAB_N ? src[ent * EV + (i % EV)] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// error-free (hi, lo) += d  (TwoSum, then renormalize)
template <typename T> __device__ __forceinline__ void acc2(T& hi, T& lo, T d)
{
    const T s = hi + d;
    const T bv = s - hi;
    const T e = (hi - (s - bv)) + (d - bv);
    const T l = lo + e;
    const T h = s + l;
    lo = l - (h - s);
    hi = h;
}

// ---------------------------------------------------------------------------
// symmetric pair schedule of the persistent kernel.  H1 and H2 depend on the
// pair distance only, and the contribution of a pair is even in d, so one
// evaluation serves both ends: target i gains Ht F_j + H2 (F_j . d) d and
// source j gains Ht F_i + H2 (F_i . d) d (eq. BrV).  Points form blocks of
// 64 (one per lane); for blocks a <= b, lane l pairs its point 64a + l with
// the point 64b + (l + s) mod 64 at offset s, s = 0..63 for a < b and
// s = 1..32 within a block (s = 32 pairs each couple twice, so lanes 32..63
// skip it).  The accumulator of the moving point rotates down one lane per
// offset.  All offsets of all block pairs (32 B^2 for B blocks) are split
// into WPS equal contiguous ranges, one per wave.  Each block is stored twice
// in a row (src2), so the point at offset s is read at lane + s.
// ---------------------------------------------------------------------------

// value of lane (l + 1) mod 64 (wave_rol:1; every lane has a source, so no
// fallback value is needed)
__device__ __forceinline__ float lane_rot(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x134, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_rot(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, 0x134, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), 0x134, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// v as an opaque wave-uniform value (a scalar register the compiler cannot
// fold into constants)
__device__ __forceinline__ int opaque_uniform(int v)
{
    int r;
    asm volatile("s_mov_b32 %0, %1" : "=s"(r) : "s"(v));
    return r;
}

// slot of point i in the doubled source array
__device__ __forceinline__ int src2_slot(int i) { return ((i >> 6) << 7) + (i & 63); }

// kernel functions of one pair at offset (dx, dy).  FP64: direct evaluation.
// FP32 (positions scaled by rho): the table (FAR = false; a pair beyond it
// gives zeros and, with CHECK, sets far), or the direct evaluation of pairs
// beyond the table only (FAR = true; zeros for the others).  H2 comes scaled
// to the coordinates (H2 / sigma in FP32).
template <typename T, bool FAR, bool CHECK = true, bool WRAP = false>
__device__ __forceinline__ void pair_kernel(const SysConst<T>& C, const char* et, T dx, T dy, T& Ht, T& H2,
                                            bool& far)
{
    if constexpr (sizeof(T) == 8) {
        kernel_eval<T>(C, fma_t(dx, dx, dy * dy), Ht, H2);
    } else {
        const uint32_t bits = __builtin_bit_cast(uint32_t, fmaf(dx, dx, fmaf(dy, dy, 1.0f)));
        const uint32_t id = bits >> TAB_SHIFT;
        if constexpr (!FAR) {
            if constexpr (CHECK) far = far || id >= TAB_END;
            if constexpr (WRAP) {
                // the index window at LDS address 0 (tab_load_window): the
                // entry's address is its offset in the window (an LDS
                // address, which only the device pass compiles)
#if defined(__HIP_DEVICE_COMPILE__)
                typedef const __attribute__((address_space(3))) TabE* LdsTabE;
                const TabE e = *(LdsTabE)(uintptr_t)tab_win_off(bits);
                tab_eval(e, tab_u(bits), Ht, H2);
#endif
            } else {
                tab_eval(*reinterpret_cast<const TabE*>(et + (min(id, TAB_END) << 5)), tab_u(bits), Ht, H2);
            }
        } else {
            Ht = 0.0f;
            H2 = 0.0f;
            if (id >= TAB_END) {
                kernel_eval<float>(C, fmaf(dx, dx, dy * dy) * C.its, Ht, H2);
                H2 *= C.its;
            }
        }
    }
}

// offsets [s_lo, s_hi) of block pair (a, b); adds the target sums to block
// a's and the moving points' sums to block b's accumulators of this lane
template <typename T, int TPL, bool FAR, bool CHECK = true, bool WRAP = false>
__device__ __forceinline__ bool sym_offsets(const SysConst<T>& C, const char* et, const Src4<T>* src2, int a, int b,
                                            int s_lo, int s_hi, int lane, T (&accx)[TPL], T (&accy)[TPL])
{
    const Src4<T> ti = src2[(a << 7) + lane];
    const Src4<T>* sp = src2 + (b << 7) + lane;
    T ax = (T)0, ay = (T)0, bx = (T)0, by = (T)0;
    bool far = false;
    // offsets every lane takes (wave-uniform: a scalar loop counter), two
    // per iteration (one address update for both loads)
    const int s_full = __builtin_amdgcn_readfirstlane((a == b) ? min(s_hi, 32) : s_hi);
    // the pair's 2x2 tensor Ht I + H2 d d^T (5 operations) applied to both
    // ends' forces (8 FMAs): 13 operations against 14 for the two dot
    // products F.d, their scaling by H2 and the four terms of each end
    auto offset = [&](const Src4<T>& q) {
        const T dx = ti.x - q.x, dy = ti.y - q.y;
        T Ht, H2;
        pair_kernel<T, FAR, CHECK, WRAP>(C, et, dx, dy, Ht, H2, far);
        const T hx = H2 * dx, hy = H2 * dy;
        const T mxx = fma_t(hx, dx, Ht), myy = fma_t(hy, dy, Ht), mxy = hx * dy;
        ax = fma_t(mxx, q.fx, fma_t(mxy, q.fy, ax));
        ay = fma_t(mxy, q.fx, fma_t(myy, q.fy, ay));
        bx = lane_rot(fma_t(mxx, ti.fx, fma_t(mxy, ti.fy, bx)));
        by = lane_rot(fma_t(mxy, ti.fx, fma_t(myy, ti.fy, by)));
    };
    int s = __builtin_amdgcn_readfirstlane(s_lo);
    for (; s + 1 < s_full; s += 2) {
        offset(sp[s]);
        offset(sp[s + 1]);
    }
    if (s < s_full) offset(sp[s]);
    if (s_full < s_hi) {
        // offset 32 within a block: lanes 32..63 repeat lanes 0..31's couples
        const Src4<T> q = sp[32];
        const T dx = ti.x - q.x, dy = ti.y - q.y;
        T Ht, H2;
        pair_kernel<T, FAR, CHECK, WRAP>(C, et, dx, dy, Ht, H2, far);
        Ht = lane < 32 ? Ht : (T)0;
        H2 = lane < 32 ? H2 : (T)0;
        const T hx = H2 * dx, hy = H2 * dy;
        const T mxx = fma_t(hx, dx, Ht), myy = fma_t(hy, dy, Ht), mxy = hx * dy;
        ax = fma_t(mxx, q.fx, fma_t(mxy, q.fy, ax));
        ay = fma_t(mxy, q.fx, fma_t(myy, q.fy, ay));
        bx = lane_rot(fma_t(mxx, ti.fx, fma_t(mxy, ti.fy, bx)));
        by = lane_rot(fma_t(mxy, ti.fx, fma_t(myy, ti.fy, by)));
    }
    // lane l now holds the sums of point (l + s_hi) mod 64 of block b
    const int from = (lane - s_hi) & 63;
    bx = __shfl(bx, from, 64);
    by = __shfl(by, from, 64);
#pragma unroll
    for (int c = 0; c < TPL; ++c) {
        if (c == a) {
            accx[c] += ax;
            accy[c] += ay;
        }
        if (c == b) {
            accx[c] += bx;
            accy[c] += by;
        }
    }
    return far;
}

// this wave's share of the pair sums of all n points: accx[c], accy[c] hold
// the partial velocity of point 64c + lane.  CHECK = false: the caller
// guarantees that no FP32 pair lies beyond the table, which then is read
// without the per-pair test (an index beyond it reads a zero entry).
// WRAP: tab points at the table's LDS index window (tab_load_window)
template <typename T, int TPL, int WPS, bool CHECK = true, bool WRAP = false>
__device__ __forceinline__ void pair_phase_sym(const SysConst<T>& C, const TabSys* tab, const Src4<T>* src2, int n,
                                               int wave, int lane, T (&accx)[TPL], T (&accy)[TPL])
{
#pragma unroll
    for (int c = 0; c < TPL; ++c) accx[c] = accy[c] = (T)0;
    const char* et = nullptr;
    if constexpr (WRAP) {
        // tab is the table's LDS index window
        et = reinterpret_cast<const char*>(tab);
    } else if constexpr (sizeof(T) == 4) {
        // entry of index id at et + (id << 5) bytes: the bias goes into a
        // wave-uniform base (a register operand of the address arithmetic;
        // gfx9 address arithmetic takes no 32-bit literal)
        et = reinterpret_cast<const char*>(tab->e) + opaque_uniform(-(int)(TAB_BIAS * sizeof(TabE)));
    }
    const int B = (n + 63) >> 6;
    const int S = 32 * B * B;
    const int per = (S + WPS - 1) / WPS;
    const int g0 = min(S, wave * per), g1 = min(S, g0 + per);
    int g = 0;  // first offset index of block pair (a, b)
    for (int a = 0; a < B && g < g1; ++a) {
        for (int b = a; b < B && g < g1; ++b) {
            const int len = (a == b) ? 32 : 64, base = (a == b) ? 1 : 0;
            const int lo = max(g0, g), hi = min(g1, g + len);
            if (lo < hi) {
                const int s_lo = lo - g + base, s_hi = hi - g + base;
                const bool far =
                    sym_offsets<T, TPL, false, CHECK, WRAP>(C, et, src2, a, b, s_lo, s_hi, lane, accx, accy);
                if constexpr (sizeof(T) == 4 && CHECK) {
                    if (__any(far)) sym_offsets<T, TPL, true>(C, et, src2, a, b, s_lo, s_hi, lane, accx, accy);
                }
            }
            g += len;
        }
    }
}

// The single block pair (a, b) and offset range [s_lo, s_hi) of this wave's
// share of pair_phase_sym's schedule for n points, when the share lies in
// one block pair (as for 128 points over 8 waves: 16 offsets each), else
// false.  Step-invariant: a run finds it once.
template <int WPS>
__device__ __forceinline__ bool sym_one_segment(int n, int wave, int& sa, int& sb, int& s_lo, int& s_hi)
{
    const int B = (n + 63) >> 6;
    const int S = 32 * B * B;
    const int per = (S + WPS - 1) / WPS;
    const int g0 = min(S, wave * per), g1 = min(S, g0 + per);
    if (g0 >= g1) return false;
    int g = 0;
    for (int a = 0; a < B; ++a) {
        for (int b = a; b < B; ++b) {
            const int len = (a == b) ? 32 : 64, base = (a == b) ? 1 : 0;
            if (g0 >= g && g1 <= g + len) {
                sa = a;
                sb = b;
                s_lo = g0 - g + base;
                s_hi = g1 - g + base;
                return true;
            }
            g += len;
        }
    }
    return false;
}

// pair_phase_sym for a wave whose share is the one segment found by
// sym_one_segment (same sums, same order)
template <typename T, int TPL, bool CHECK = true, bool WRAP = false>
__device__ __forceinline__ void pair_phase_seg(const SysConst<T>& C, const TabSys* tab, const Src4<T>* src2, int a,
                                               int b, int s_lo, int s_hi, int lane, T (&accx)[TPL], T (&accy)[TPL])
{
#pragma unroll
    for (int c = 0; c < TPL; ++c) accx[c] = accy[c] = (T)0;
    const char* et = nullptr;
    if constexpr (WRAP) {
        et = reinterpret_cast<const char*>(tab);
    } else if constexpr (sizeof(T) == 4) {
        et = reinterpret_cast<const char*>(tab->e) + opaque_uniform(-(int)(TAB_BIAS * sizeof(TabE)));
    }
    const bool far = sym_offsets<T, TPL, false, CHECK, WRAP>(C, et, src2, a, b, s_lo, s_hi, lane, accx, accy);
    if constexpr (sizeof(T) == 4 && CHECK) {
        if (__any(far)) sym_offsets<T, TPL, true>(C, et, src2, a, b, s_lo, s_hi, lane, accx, accy);
    }
}

// sum over the 64 lanes of a wavefront (butterfly; lane j's result is
// deterministic)
template <typename T> __device__ __forceinline__ T wave_total(T v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Whether the tail schedule below does less work than the padded symmetric
// one for n points: r tail points (n = 64 Bf + r, 0 < r < 64) cost about
// r (33 Bf + 52) lane-operations per lane against 33 for each of the
// 32 (2 Bf + 1) offsets the padded last block adds.
__host__ __device__ constexpr bool tail_pays(int n)
{
    const int Bf = n >> 6, r = n & 63;
    return r != 0 && r * (33 * Bf + 52) < 33 * 32 * (2 * Bf + 1);
}

// Pair sums of n points whose last block is partly filled (r = n - 64 Bf
// points, 0 < r < 64): the symmetric schedule covers the Bf full blocks,
// and the r tail points take their pairs point by point instead of as a
// padded block of 64:
//  * tail point j against full block a: lane l evaluates the pair
//    (64 a + l, tail j) once; point 64 a + l keeps its share, and the
//    shares of tail point j, summed over all full blocks in each lane, are
//    summed over the wavefront once and kept by lane j;
//  * tail point j as a source within the tail: lanes l < r take the pair
//    (tail l, tail j) for target tail l only.
// Every ordered pair is taken once.  The full blocks' offsets are split
// over the waves as in pair_phase_sym; tail point j goes to wave j mod WPS.
// seg: this wave's share of the full blocks' schedule as found by
// sym_one_segment for 64 Bf points (seg[0] != 0: a single segment a = seg[1],
// b = seg[2], offsets [seg[3], seg[4])), or null
template <typename T, int TPL, int WPS>
__device__ __forceinline__ void pair_phase_tail(const SysConst<T>& C, const TabSys* tab, const Src4<T>* src2, int n,
                                                int wave, int lane, T (&accx)[TPL], T (&accy)[TPL],
                                                const int* seg = nullptr)
{
    const int Bf = n >> 6, r = n & 63;
    if (seg && seg[0])
        pair_phase_seg<T, TPL>(C, tab, src2, seg[1], seg[2], seg[3], seg[4], lane, accx, accy);
    else
        pair_phase_sym<T, TPL, WPS>(C, tab, src2, 64 * Bf, wave, lane, accx, accy);
    const char* et = nullptr;
    if constexpr (sizeof(T) == 4)
        et = reinterpret_cast<const char*>(tab->e) + opaque_uniform(-(int)(TAB_BIAS * sizeof(TabE)));
    const bool tl_live = lane < r;
    const Src4<T> tp = src2[src2_slot(64 * Bf + (tl_live ? lane : r - 1))];
    for (int j = wave; j < r; j += WPS) {
        const Src4<T> q = src2[src2_slot(64 * Bf + j)];
        T bx = (T)0, by = (T)0;
        bool far = false;
        // one pass over tail point j's pairs; FAR selects the direct
        // evaluation of pairs beyond the FP32 table (zeros for the others)
        auto pass = [&](auto far_tag) {
            constexpr bool FAR = decltype(far_tag)::value;
#pragma unroll
            for (int a = 0; a < TPL; ++a) {
                if (a < Bf) {
                    const Src4<T> ti = src2[(a << 7) + lane];
                    const T dx = ti.x - q.x, dy = ti.y - q.y;
                    T Ht, H2;
                    pair_kernel<T, FAR>(C, et, dx, dy, Ht, H2, far);
                    const T hx = H2 * dx, hy = H2 * dy;
                    const T mxx = fma_t(hx, dx, Ht), myy = fma_t(hy, dy, Ht), mxy = hx * dy;
                    accx[a] = fma_t(mxx, q.fx, fma_t(mxy, q.fy, accx[a]));
                    accy[a] = fma_t(mxy, q.fx, fma_t(myy, q.fy, accy[a]));
                    bx = fma_t(mxx, ti.fx, fma_t(mxy, ti.fy, bx));
                    by = fma_t(mxy, ti.fx, fma_t(myy, ti.fy, by));
                }
            }
            const T dx = tp.x - q.x, dy = tp.y - q.y;
            T Ht, H2;
            pair_kernel<T, FAR>(C, et, dx, dy, Ht, H2, far);
            Ht = tl_live ? Ht : (T)0;
            H2 = tl_live ? H2 : (T)0;
            const T fdj = H2 * fma_t(q.fx, dx, q.fy * dy);
#pragma unroll
            for (int c = 0; c < TPL; ++c) {
                if (c == Bf) {
                    accx[c] = fma_t(Ht, q.fx, fma_t(fdj, dx, accx[c]));
                    accy[c] = fma_t(Ht, q.fy, fma_t(fdj, dy, accy[c]));
                }
            }
        };
        pass(std::integral_constant<bool, false>());
        if constexpr (sizeof(T) == 4) {
            if (__any(far)) pass(std::integral_constant<bool, true>());
        }
        bx = wave_total(bx);
        by = wave_total(by);
#pragma unroll
        for (int c = 0; c < TPL; ++c) {
            if (c == Bf && lane == j) {
                accx[c] += bx;
                accy[c] += by;
            }
        }
    }
}

}  // namespace swim
