// Device code of the ES-BGK stream-collide step for gfx950 (MI355X).
//
// Data layout (per population set f or g): Q planes of ncell values, plane i
// holding direction i of the lattice's storage order, cells x-fastest.  Each
// value is stored as a deviation from the rest state scaled by a per-shell
// power of two s = 2^k (k = floor(log2(1/w))):
//     F_i = s_i (f_i - w_i),     E_i = s_i (g_i - w_i N_f/2)
// (rho0 = T0 = 1), in FP32, FP16 or BF16.  Scaling by a power of two is exact,
// so FP32 results equal those of unscaled deviations; in FP16/BF16 it keeps
// the small-weight directions in the normal range.  FP16/BF16 domains with
// both populations keep F_i and E_i side by side in one 4-byte element of a
// single set (kPaired).
//
// Streaming uses the A-A pattern in place: after an even number of steps
// f_i(x) sits at (x, plane i); after an odd number it sits at
// (x - c_i, plane opp(i)).  The even kernel reads the own cell's planes i and
// writes plane opp(i); the odd kernel reads (x - c, plane -c) and (x + c,
// plane +c) and writes the same two locations with the post-collision values
// of +c and -c.  Each thread reads and writes exactly the same set of
// locations, so the update is race-free without a second buffer.  The
// two-copy pull scheme (LAY_PULL) reads (x - c_i, plane i) of one copy and
// writes (x, plane i) of the other: the same arithmetic on the same values,
// with whole aligned cache lines stored.
//
// The collision (Section V of the paper) per cell, in FP32 registers:
//   moments rho, j, second moment -> u, sigma, T_tr, T_int, T_eq, T_rel;
//   A = Lambda - delta with Lambda = (1-kappa)[(1-nu)T_tr delta + nu sigma]
//       + kappa T_eq delta;
//   target G_i = w_i rho (E_i +- O_i) from the general-term coefficients
//   a^(1..4) contracted with H^(1..4)(xi_i), written through the invariants
//   s1 = u.xi, a = xi.A.xi, b = u.A.xi, c = xi.A^2.xi, t = tr A, U = u.u,
//   m = u.A.u, q = A:A per velocity pair +-xi (E even, O odd in xi):
//     E - 1 = h/2 + h^2/8 - s1^4/12 - c/2 - b s1 + q/4 + m/2,  h = a - t - U + s1^2
//     O     = s1 (1 + (a - t - U)/2 + s1^2/6) - b
//   (the sum of a^(n).H^(n)/n! for n <= 4 of Eq. GExpansion);
//   relax f toward G and g toward (N_f/2) T_rel G at rate omega; then restore
//   the pre-collision mass and momentum exactly in FP32 (a projection that is
//   identically zero in exact arithmetic and removes the drift that FP32
//   rounding of the lattice constants would otherwise cause).
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "lattice.hpp"

namespace esbgk {

enum { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

template <int S>
struct StoreBytes {
    static constexpr uint32_t value = S == ST_F32 ? 4u : 2u;
};

// FP16/BF16 storage of a domain with both populations keeps f_i and g_i of a
// cell side by side in one 4-byte element (f in the low half): one load and
// one store per direction instead of two, and half as many address streams.
// FP32 keeps separate f and g sets (its paired 8-byte elements measured
// slower).
template <int S, bool HAS_G>
inline constexpr bool kPaired = S != ST_F32 && HAS_G;

// bytes from one cell's element to the next in a plane
template <int S, bool HAS_G>
inline constexpr uint32_t kElemBytes = kPaired<S, HAS_G> ? 2 * StoreBytes<S>::value : StoreBytes<S>::value;

// --------------------------------------------------------------------------
// Small helpers
// --------------------------------------------------------------------------

// n / d for n < 2^31 with a precomputed multiplier (round-up method):
// s = ceil(log2 d), m = floor(2^32 (2^s - d)/d) + 1, q = (umulhi(n, m) + n) >> s.
struct FastDiv {
    uint32_t d, m, s;
};

__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) { return (__umulhi(n, f.m) + n) >> f.s; }

struct Geom {
    uint32_t nx, ny, nz, ncell;
    FastDiv by_nx, by_nxy;
};

// Collision constants of one domain (FP32).  The constants that multiply
// first-order deviations in the moments and the target (r^2, 2/N_f and the
// weights) also carry their FP32 rounding error as a second float (_lo):
// rounded once, they would make the FP32 scheme a slightly different
// lattice (sound speed off by a few 1e-8), an error that grows linearly
// with the acoustic phase travelled.
struct Coll {
    float omega;        // heat-flux (collision) rate
    float kappa, nu;    // Lambda / T_rel blend and ES parameter
    float r2, r2_lo;    // r^2 (xi = r c)
    float hN;           // N_f / 2
    float two_over_nf, two_over_nf_lo;   // 2 / N_f (0 when N_f = 0)
    float cD, cN;       // D/(D+N_f), N_f/(D+N_f)
    float wh[MAX_SHELL];   // s w per shell
    float wl[MAX_SHELL];   // s w - wh per shell
    float isc[MAX_SHELL];  // 1/s per shell
};

// x * (hi + lo) with the product of the two-float constant formed exactly
// up to the final rounding
__device__ __forceinline__ float mul2(float x, float hi, float lo) { return __builtin_fmaf(x, hi, x * lo); }
template <class R>
__device__ __forceinline__ R mul_r2(R x, float hi, float lo) {
    if constexpr (sizeof(R) == 8) return x * (double(hi) + double(lo));
    else return __builtin_fmaf(x, hi, x * lo);
}

template <int C, class T>
__device__ __forceinline__ T acc_c(T acc, T v) {
    if constexpr (C == 0) return acc;
    else if constexpr (C == 1) return acc + v;
    else if constexpr (C == -1) return acc - v;
    else if constexpr (sizeof(T) == 8) return __builtin_fma(T(C), v, acc);
    else return __builtin_fmaf(T(C), v, acc);
}

template <int C>
__device__ __forceinline__ float mul_c(float v) {
    if constexpr (C == 1) return v;
    else if constexpr (C == -1) return -v;
    else return float(C) * v;
}

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}

template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <class L, int P>
constexpr bool first_in_shell() { return P == 0 || L::P[P - 1].shell != L::P[P].shell; }
template <class L, int P>
constexpr bool last_in_shell() { return P == L::NP - 1 || L::P[P + 1].shell != L::P[P].shell; }

// --------------------------------------------------------------------------
// Storage codecs over buffer resources.  One resource spans a whole
// population set (all Q planes, at most 4 GiB); the plane is selected by the
// scalar offset plane * plane_bytes, the cell by the per-lane offset.  Reads
// past the set return 0 and stores past it are dropped.
// --------------------------------------------------------------------------

__device__ __forceinline__ __amdgpu_buffer_rsrc_t set_rsrc(char *base, uint32_t set_bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)set_bytes, 0x00020000);
}

// CP: cache-policy bits of the buffer instruction (0 = default, 2 = streaming
// / non-temporal).
template <int S, int CP = 0>
__device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    if constexpr (S == ST_F32) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, CP));
    } else if constexpr (S == ST_F16) {
        unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, (int)soff, CP);
        float v = __half2float(__ushort_as_half(h));
        // keep the converted value in one register: without this the compiler
        // folds some conversions into mixed-precision FMAs and keeps both the
        // FP16 and FP32 copies alive (about 70 more VGPRs)
        asm("" : "+v"(v));
        return v;
    } else {
        unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, (int)soff, CP);
        return __uint_as_float(uint32_t(h) << 16);
    }
}

template <int S, int CP = 0>
__device__ __forceinline__ void st(float v, __amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    if constexpr (S == ST_F32) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, (int)soff, CP);
    } else if constexpr (S == ST_F16) {
        // round to FP32 first, then to FP16, in every kernel: otherwise the
        // compiler may fuse the last FMA with the conversion (one rounding)
        // in some kernels and not in others, and two paths that compute the
        // same step would store different bits
        asm("" : "+v"(v));
        __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v)), r, (int)off, (int)soff, CP);
    } else {
        __builtin_amdgcn_raw_buffer_store_b16(__bfloat16_as_ushort(__float2bfloat16(v)), r, (int)off, (int)soff, CP);
    }
}

// f and g of one paired 4-byte element (FP16/BF16 storage only).
template <int S, int CP = 0>
__device__ __forceinline__ void ld_pair(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff, float &f, float &g) {
    static_assert(S != ST_F32, "paired elements hold 2-byte values");
    const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, CP);
    if constexpr (S == ST_F16) {
        f = __half2float(__ushort_as_half((unsigned short)(v & 0xffffu)));
        g = __half2float(__ushort_as_half((unsigned short)(v >> 16)));
        asm("" : "+v"(f));   // see ld
        asm("" : "+v"(g));
    } else {
        f = __uint_as_float(v << 16);
        g = __uint_as_float(v & 0xffff0000u);
    }
}

template <int S, int CP = 0>
__device__ __forceinline__ void st_pair(float f, float g, __amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    static_assert(S != ST_F32, "paired elements hold 2-byte values");
    // both halves in one packed round-to-nearest-even conversion
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    uint32_t v;
    if constexpr (S == ST_F16) {
        asm("" : "+v"(f));   // see st
        asm("" : "+v"(g));
        typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
        v = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){f, g}, f16x2));
    } else {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        v = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){f, g}, bf16x2));
    }
    __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)off, (int)soff, CP);
}

// The two population sets of a domain as buffer resources.  With paired
// elements g is the same storage as f shifted by 2 bytes (the high half), so
// that per-population element accesses work unchanged.
struct Sets {
    __amdgpu_buffer_rsrc_t f, g;
    uint32_t pb;   // bytes per plane
    __device__ __forceinline__ Sets(char *fb, char *gb, uint32_t plane_bytes, uint32_t set_bytes)
        : f(set_rsrc(fb, set_bytes)), g(set_rsrc(gb ? gb : fb, set_bytes)), pb(plane_bytes) {}
    __device__ __forceinline__ uint32_t so(int plane) const { return uint32_t(plane) * pb; }
};

// --------------------------------------------------------------------------
// Neighbour offsets: wrapped coordinates of x + k for |k| <= REACH, as byte
// offsets, so that the location x + c costs one or two adds.  A location is
// a per-lane byte offset plus a wave-uniform one (added to the plane's
// scalar offset).
// --------------------------------------------------------------------------

struct Off {
    uint32_t v;   // per-lane byte offset
    uint32_t s;   // wave-uniform byte offset
};

// B: bytes per cell element (kElemBytes).
template <class L, uint32_t B>
struct Nbr {
    static constexpr int R = L::REACH;
    uint32_t xo[2 * R + 1], yo[2 * R + 1], zo[L::D == 3 ? 2 * R + 1 : 1];
    uint32_t own;

    __device__ __forceinline__ void init(uint32_t cell, const Geom &g) {
        uint32_t x, y, z = 0;
        if constexpr (L::D == 2) {
            y = fdiv(cell, g.by_nx);
            x = cell - y * g.nx;
        } else {
            z = fdiv(cell, g.by_nxy);
            uint32_t rem = cell - z * (g.nx * g.ny);
            y = fdiv(rem, g.by_nx);
            x = rem - y * g.nx;
        }
        own = cell * B;
        static_for<2 * R + 1>([&](auto kk) {
            constexpr int k = decltype(kk)::value - R;
            int xv = int(x) + k, yv = int(y) + k;
            if constexpr (k < 0) {
                xv = xv < 0 ? xv + int(g.nx) : xv;
                yv = yv < 0 ? yv + int(g.ny) : yv;
            } else if constexpr (k > 0) {
                xv = xv >= int(g.nx) ? xv - int(g.nx) : xv;
                yv = yv >= int(g.ny) ? yv - int(g.ny) : yv;
            }
            xo[k + R] = uint32_t(xv) * B;
            yo[k + R] = uint32_t(yv) * (g.nx * B);
            if constexpr (L::D == 3) {
                int zv = int(z) + k;
                if constexpr (k < 0) zv = zv < 0 ? zv + int(g.nz) : zv;
                else if constexpr (k > 0) zv = zv >= int(g.nz) ? zv - int(g.nz) : zv;
                zo[k + R] = uint32_t(zv) * (g.nx * g.ny * B);
            }
        });
    }

    __device__ __forceinline__ Off self() const { return {own, 0u}; }

    template <int CX, int CY, int CZ>
    __device__ __forceinline__ Off at() const {
        if constexpr (L::D == 2) return {xo[CX + R] + yo[CY + R], 0u};
        else return {xo[CX + R] + yo[CY + R] + zo[CZ + R], 0u};
    }
};

// Row-wave addressing, for domains whose x-rows are whole waves (nx a
// multiple of 64, waves starting at multiples of 64 cells).  y and z are the
// same on all lanes of a wave, so their offsets are scalar.  In a wave that
// does not touch x = 0 or x = nx - 1 ("inner"), x + k never wraps: the x
// offset is one register plus the instruction's immediate (k + R) B.  Waves
// at the two ends of a row wrap x per lane (RowView<.., false>).
template <class L, uint32_t B, bool INNER>
struct RowView {
    static constexpr int R = L::REACH;
    uint32_t xb;                                   // (x - R) B, per lane
    uint32_t nxB;                                  // nx B
    uint32_t yo[2 * R + 1], zo[L::D == 3 ? 2 * R + 1 : 1];   // uniform

    template <int CY, int CZ>
    __device__ __forceinline__ uint32_t yz() const {
        if constexpr (L::D == 2) return yo[CY + R];
        else return yo[CY + R] + zo[CZ + R];
    }
    template <int CX>
    __device__ __forceinline__ uint32_t xoff() const {
        if constexpr (INNER || CX == 0) {
            return xb + uint32_t((CX + R) * int(B));
        } else {
            const uint32_t v = xb + uint32_t((CX + R) * int(B));   // (x + CX) B, unwrapped
            if constexpr (CX < 0) return int32_t(v) < 0 ? v + nxB : v;
            else return v >= nxB ? v - nxB : v;
        }
    }
    __device__ __forceinline__ Off self() const { return {xoff<0>(), yz<0, 0>()}; }
    template <int CX, int CY, int CZ>
    __device__ __forceinline__ Off at() const { return {xoff<CX>(), yz<CY, CZ>()}; }
};

template <class L, uint32_t B>
struct RowNbr {
    static constexpr int R = L::REACH;
    RowView<L, B, true> v;
    bool inner;

    __device__ __forceinline__ void init(uint32_t cell, const Geom &g) {
        const uint32_t c0 = __builtin_amdgcn_readfirstlane(cell);   // first cell of the wave
        uint32_t y, z = 0, x0;
        if constexpr (L::D == 2) {
            y = fdiv(c0, g.by_nx);
            x0 = c0 - y * g.nx;
        } else {
            z = fdiv(c0, g.by_nxy);
            const uint32_t rem = c0 - z * (g.nx * g.ny);
            y = fdiv(rem, g.by_nx);
            x0 = rem - y * g.nx;
        }
        inner = x0 != 0 && x0 + 64 < g.nx;
        v.xb = (cell - c0 + x0) * B - uint32_t(R) * B;
        v.nxB = g.nx * B;
        static_for<2 * R + 1>([&](auto kk) {
            constexpr int k = decltype(kk)::value - R;
            int yv = int(y) + k;
            if constexpr (k < 0) yv = yv < 0 ? yv + int(g.ny) : yv;
            else if constexpr (k > 0) yv = yv >= int(g.ny) ? yv - int(g.ny) : yv;
            v.yo[k + R] = uint32_t(yv) * (g.nx * B);
            if constexpr (L::D == 3) {
                int zv = int(z) + k;
                if constexpr (k < 0) zv = zv < 0 ? zv + int(g.nz) : zv;
                else if constexpr (k > 0) zv = zv >= int(g.nz) ? zv - int(g.nz) : zv;
                v.zo[k + R] = uint32_t(zv) * (g.nx * g.ny * B);
            }
        });
    }
    // the wrapping view; its per-lane base passes through an empty asm so that
    // the wrapped offsets are recomputed where they are used instead of being
    // kept alive across the collision
    __device__ __forceinline__ RowView<L, B, false> edge() const {
        RowView<L, B, false> e;
        e.xb = v.xb;
        asm volatile("" : "+v"(e.xb));
        e.nxB = v.nxB;
        for (int k = 0; k < 2 * R + 1; k++) e.yo[k] = v.yo[k];
        if constexpr (L::D == 3)
            for (int k = 0; k < 2 * R + 1; k++) e.zo[k] = v.zo[k];
        return e;
    }
};

// --------------------------------------------------------------------------
// Gather / scatter of all populations of one cell.  Layouts of the stored
// state (where the value of direction i at cell x lives):
//   LAY_EVEN: (x, plane i)             A-A, after an even number of steps
//   LAY_ODD : (x - c_i, plane opp(i))  A-A, after an odd number of steps
//   LAY_PULL: (x - c_i, plane i)       two-copy pull, every step; these are
//             the post-collision values not yet streamed
// --------------------------------------------------------------------------

enum : int { LAY_EVEN = 0, LAY_ODD = 1, LAY_PULL = 2 };

template <class L, int S, int LAY, bool HAS_G, int CP = 0, class NB>
__device__ __forceinline__ void gather(const Sets &R, const NB &nb, float *F, float *E) {
    constexpr bool PAIR = kPaired<S, HAS_G>;
    // f and g of direction i at byte offsets (v, s) of plane `plane`
    auto load = [&](int i, int plane, uint32_t v, uint32_t s) __attribute__((always_inline)) {
        if constexpr (PAIR) {
            ld_pair<S, CP>(R.f, v, R.so(plane) + s, F[i], E[i]);
        } else {
            F[i] = ld<S, CP>(R.f, v, R.so(plane) + s);
            if constexpr (HAS_G) E[i] = ld<S, CP>(R.g, v, R.so(plane) + s);
        }
    };
    const Off o = nb.self();
    load(0, 0, o.v, o.s);
    static_for<L::NP>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        constexpr int cx = L::P[p].c[0], cy = L::P[p].c[1], cz = L::P[p].c[2];
        constexpr int a = 2 * p + 1, b = 2 * p + 2;   // c_b = -c_a
        if constexpr (LAY == LAY_EVEN) {
            load(a, a, o.v, o.s);
            load(b, b, o.v, o.s);
        } else {
            // direction a comes from x - c_a, direction b from x + c_a
            constexpr int pa = LAY == LAY_ODD ? b : a, pb = LAY == LAY_ODD ? a : b;
            const Off op = nb.template at<cx, cy, cz>();
            const Off om = nb.template at<-cx, -cy, -cz>();
            load(a, pa, om.v, om.s);
            load(b, pb, op.v, op.s);
        }
    });
}

// Write post-collision populations of a cell whose state was read in layout
// LAY.  A-A flips the parity in place: after LAY_EVEN, f*_i goes to the own
// cell's plane opp(i); after LAY_ODD, to (x + c_i, plane i).  LAY_PULL
// writes f*_i to the own cell's plane i of the other copy (aligned, whole
// cache lines), which is LAY_PULL again.
template <class L, int S, int LAY, bool HAS_G, int CP = 0, class NB>
__device__ __forceinline__ void scatter(const Sets &R, const NB &nb, const float *F, const float *E) {
    constexpr bool PAIR = kPaired<S, HAS_G>;
    auto store = [&](int i, int plane, uint32_t v, uint32_t s) __attribute__((always_inline)) {
        if constexpr (PAIR) {
            st_pair<S, CP>(F[i], E[i], R.f, v, R.so(plane) + s);
        } else {
            st<S, CP>(F[i], R.f, v, R.so(plane) + s);
            if constexpr (HAS_G) st<S, CP>(E[i], R.g, v, R.so(plane) + s);
        }
    };
    const Off o = nb.self();
    store(0, 0, o.v, o.s);
    static_for<L::NP>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        constexpr int cx = L::P[p].c[0], cy = L::P[p].c[1], cz = L::P[p].c[2];
        constexpr int a = 2 * p + 1, b = 2 * p + 2;
        if constexpr (LAY == LAY_ODD) {
            const Off op = nb.template at<cx, cy, cz>();
            const Off om = nb.template at<-cx, -cy, -cz>();
            store(a, a, op.v, op.s);
            store(b, b, om.v, om.s);
        } else {
            constexpr int pa = LAY == LAY_EVEN ? b : a, pb = LAY == LAY_EVEN ? a : b;
            store(a, pa, o.v, o.s);
            store(b, pb, o.v, o.s);
        }
    });
}

// --------------------------------------------------------------------------
// Per-cell macroscopic state and the Gaussian target.
// --------------------------------------------------------------------------

template <int D>
struct CellState {
    float drho, rho, irho;
    float J[3];      // lattice-unit momentum sum c d (j = r J)
    float M[6];      // lattice-unit central second moment S - J J^T/rho (xx, xy, xz, yy, yz, zz)
    float Ttr1, Tint1, Teq1, Trel1;   // temperatures minus one
};

// Invariants of the target: with Ah = r^2 A, uh = r^2 u/r (= r^2 J/rho in
// lattice form), the per-direction quantities are dot products with the
// integer velocity c.  R is the precision the target is evaluated in: FP64
// with FP32 storage (in FP32 the rounding of the target leaves a bias that a
// weakly damped acoustic or entropy wave integrates over thousands of steps,
// a few 1e-8 absolute in rho and u after 5000 steps; in FP64 that part is
// 1e-10, for about 600 FP64 operations per cell on a kernel bound by HBM),
// FP32 with FP16/BF16 storage, whose rounding dominates anyway.
template <int D, class R>
struct TargetInv {
    R uh[3];     // s1 = uh . c
    R Ah[6];     // a = c . Ah . c
    R wv[3];     // b = wv . c
    R A2[6];     // c4 = c . A2 . c
    R tU;        // t + U
    R K24;       // q/4 + m/2
};

template <int S>
using TargetReal = std::conditional_t<S == ST_F32, double, float>;

template <class R>
__device__ __forceinline__ R fma_r(R a, R b, R c) {
    if constexpr (sizeof(R) == 8) return __builtin_fma(a, b, c);
    else return __builtin_fmaf(a, b, c);
}

__device__ __forceinline__ int sym_idx(int a, int b) {
    // (0,0)->0 (0,1)->1 (0,2)->2 (1,1)->3 (1,2)->4 (2,2)->5
    return a <= b ? (a == 0 ? b : (a == 1 ? 2 + b : 5)) : (b == 0 ? a : (b == 1 ? 2 + a : 5));
}

// Target invariants from A (physical, symmetric, 6 slots) and the
// lattice-unit velocity ut = J/rho; r^2 = r2_hi + r2_lo.
template <int D, class R, class In = float>
__device__ __forceinline__ TargetInv<D, R> target_inv(const In *Af, const In *utf, float r2_hi, float r2_lo) {
    TargetInv<D, R> T;
    R A[6], ut[3];
#pragma unroll
    for (int k = 0; k < 6; k++) A[k] = Af[k];
#pragma unroll
    for (int k = 0; k < 3; k++) ut[k] = utf[k];
    R t = 0, U = 0, q = 0, m = 0;
    R Au[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; a++) {
        t += A[sym_idx(a, a)];
        U += ut[a] * ut[a];
#pragma unroll
        for (int b = 0; b < D; b++) Au[a] += A[sym_idx(a, b)] * ut[b];
    }
#pragma unroll
    for (int a = 0; a < D; a++) {
        m += ut[a] * Au[a];
        T.uh[a] = mul_r2(ut[a], r2_hi, r2_lo);   // first order in u
        T.wv[a] = R(r2_hi) * Au[a];
    }
#pragma unroll
    for (int a = 0; a < D; a++)
#pragma unroll
        for (int b = a; b < D; b++) {
            R s = 0;
#pragma unroll
            for (int k = 0; k < D; k++) s += A[sym_idx(a, k)] * A[sym_idx(k, b)];
            T.A2[sym_idx(a, b)] = R(r2_hi) * s;
            T.Ah[sym_idx(a, b)] = mul_r2(A[sym_idx(a, b)], r2_hi, r2_lo);   // first order in A
            q += (a == b ? R(1) : R(2)) * A[sym_idx(a, b)] * A[sym_idx(a, b)];
        }
    U *= R(r2_hi);
    m *= R(r2_hi);
    T.tU = t + U;
    T.K24 = R(0.25) * q + R(0.5) * m;
    return T;
}

// E - 1 and O for the velocity pair +-c (c compile-time).
template <int D, int CX, int CY, int CZ, class R>
__device__ __forceinline__ void target_pair(const TargetInv<D, R> &T, R &Em1, R &O) {
    R s1 = 0, a = 0, b = 0, c4 = 0;
    s1 = acc_c<CX>(s1, T.uh[0]);
    s1 = acc_c<CY>(s1, T.uh[1]);
    b = acc_c<CX>(b, T.wv[0]);
    b = acc_c<CY>(b, T.wv[1]);
    a = acc_c<CX * CX>(a, T.Ah[0]);
    a = acc_c<2 * CX * CY>(a, T.Ah[1]);
    a = acc_c<CY * CY>(a, T.Ah[3]);
    c4 = acc_c<CX * CX>(c4, T.A2[0]);
    c4 = acc_c<2 * CX * CY>(c4, T.A2[1]);
    c4 = acc_c<CY * CY>(c4, T.A2[3]);
    if constexpr (D == 3) {
        s1 = acc_c<CZ>(s1, T.uh[2]);
        b = acc_c<CZ>(b, T.wv[2]);
        a = acc_c<2 * CX * CZ>(a, T.Ah[2]);
        a = acc_c<2 * CY * CZ>(a, T.Ah[4]);
        a = acc_c<CZ * CZ>(a, T.Ah[5]);
        c4 = acc_c<2 * CX * CZ>(c4, T.A2[2]);
        c4 = acc_c<2 * CY * CZ>(c4, T.A2[4]);
        c4 = acc_c<CZ * CZ>(c4, T.A2[5]);
    }
    const R al = a - T.tU;
    const R s2 = s1 * s1;
    const R h = al + s2;
    R e = h * fma_r(R(0.125), h, R(0.5));
    e = fma_r(-s2 * R(1.0 / 12.0), s2, e);
    e = fma_r(R(-0.5), c4, e);
    e = fma_r(-b, s1, e);
    Em1 = e + T.K24;
    const R k = fma_r(s2, R(1.0 / 6.0), fma_r(R(0.5), al, R(1)));
    O = fma_r(s1, k, -b);
}

// Rest-direction E - 1 (c = 0).
template <int D, class R>
__device__ __forceinline__ R target_rest(const TargetInv<D, R> &T) {
    const R h = -T.tU;
    return h * fma_r(R(0.125), h, R(0.5)) + T.K24;
}

// w (rho (E - 1) + drho) and w rho O, w = wh + wl.
template <class R>
__device__ __forceinline__ R target_x(R Em1, float rho, float drho, float wh, float wl) {
    const R t = fma_r(R(rho), Em1, R(drho));
    return fma_r(R(wh), t, R(wl) * t);
}
template <class R>
__device__ __forceinline__ R target_y(R O, float rho, float wh, float wl) {
    const R t = R(rho) * O;
    return fma_r(R(wh), t, R(wl) * t);
}

// --------------------------------------------------------------------------
// Moments of one cell (scaled deviations in F, E).
// --------------------------------------------------------------------------

template <class L, bool HAS_G>
__device__ __forceinline__ CellState<L::D> cell_moments(const Coll &cp, const float *F, const float *E) {
    constexpr int D = L::D;
    CellState<D> cs;
    float drho = F[0] * cp.isc[0];
    float J[3] = {0, 0, 0}, S[6] = {0, 0, 0, 0, 0, 0};
    float sg = HAS_G ? E[0] * cp.isc[0] : 0.f;
    float m0 = 0, j0 = 0, j1 = 0, j2 = 0, s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0, g0 = 0;
    static_for<L::NP>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        constexpr int cx = L::P[p].c[0], cy = L::P[p].c[1], cz = L::P[p].c[2];
        constexpr int sh = L::P[p].shell;
        if constexpr (first_in_shell<L, p>()) {
            m0 = j0 = j1 = j2 = s0 = s1 = s2 = s3 = s4 = s5 = g0 = 0;
        }
        const float fa = F[2 * p + 1], fb = F[2 * p + 2];
        const float sp = fa + fb, dp = fa - fb;
        m0 += sp;
        j0 = acc_c<cx>(j0, dp);
        j1 = acc_c<cy>(j1, dp);
        s0 = acc_c<cx * cx>(s0, sp);
        s1 = acc_c<cx * cy>(s1, sp);
        s3 = acc_c<cy * cy>(s3, sp);
        if constexpr (D == 3) {
            j2 = acc_c<cz>(j2, dp);
            s2 = acc_c<cx * cz>(s2, sp);
            s4 = acc_c<cy * cz>(s4, sp);
            s5 = acc_c<cz * cz>(s5, sp);
        }
        if constexpr (HAS_G) g0 += E[2 * p + 1] + E[2 * p + 2];
        if constexpr (last_in_shell<L, p>()) {
            const float is = cp.isc[sh];
            drho = __builtin_fmaf(m0, is, drho);
            J[0] = __builtin_fmaf(j0, is, J[0]);
            J[1] = __builtin_fmaf(j1, is, J[1]);
            S[0] = __builtin_fmaf(s0, is, S[0]);
            S[1] = __builtin_fmaf(s1, is, S[1]);
            S[3] = __builtin_fmaf(s3, is, S[3]);
            if constexpr (D == 3) {
                J[2] = __builtin_fmaf(j2, is, J[2]);
                S[2] = __builtin_fmaf(s2, is, S[2]);
                S[4] = __builtin_fmaf(s4, is, S[4]);
                S[5] = __builtin_fmaf(s5, is, S[5]);
            }
            if constexpr (HAS_G) sg = __builtin_fmaf(g0, is, sg);
        }
    });
    cs.drho = drho;
    cs.rho = 1.0f + drho;
    // the temperatures and the central second moment are formed in FP64 from
    // the FP32 sums (the subtractions of the density term cancel most of the
    // sums; rounded in FP32 they bias the pressure of long waves)
    const double irho = 1.0 / (1.0 + double(drho));
    cs.irho = float(irho);
#pragma unroll
    for (int a = 0; a < 3; a++) cs.J[a] = a < D ? J[a] : 0.f;
    double trM = 0;
#pragma unroll
    for (int a = 0; a < D; a++)
#pragma unroll
        for (int b = a; b < D; b++) {
            const int k = sym_idx(a, b);
            const double Mk = double(S[k]) - double(cs.J[a]) * double(cs.J[b]) * irho;
            cs.M[k] = float(Mk);
            if (a == b) trM += Mk;
        }
    const double r2 = double(cp.r2) + double(cp.r2_lo);
    cs.Ttr1 = float((r2 * trM - double(D) * double(drho)) * irho * (1.0 / double(D)));
    if constexpr (HAS_G) {
        const double tnf = double(cp.two_over_nf) + double(cp.two_over_nf_lo);
        cs.Tint1 = float((tnf * double(sg) - double(drho)) * irho);
    } else {
        cs.Tint1 = cs.Ttr1;
    }
    // blends written so that equal temperatures pass through unchanged
    // whatever the rounding of the blend weights (cD + cN = 1 and
    // kappa + (1 - kappa) = 1 only in exact arithmetic)
    cs.Teq1 = __builtin_fmaf(cp.cN, cs.Tint1 - cs.Ttr1, cs.Ttr1);
    cs.Trel1 = __builtin_fmaf(cp.kappa, cs.Teq1 - cs.Tint1, cs.Tint1);
    return cs;
}

// A = Lambda - delta from the cell state, written as
//   [T_tr - 1 + kappa (T_eq - T_tr)] delta + (1 - kappa) nu (sigma - T_tr delta)
// (equal to (1-kappa)[(1-nu) T_tr delta + nu sigma] + kappa T_eq delta - delta),
// so that the isotropic part has coefficient one exactly and the rounding of
// the blend weights only touches the trace-free stress.  sigma - delta =
// r^2 M / rho - delta drho / rho.
template <int D>
__device__ __forceinline__ void lambda_minus_delta(const Coll &cp, const CellState<D> &cs, float *A) {
    const float beta = (1.0f - cp.kappa) * cp.nu;
    float sd[6];   // sigma - delta
#pragma unroll
    for (int k = 0; k < 6; k++) sd[k] = mul2(cs.M[k], cp.r2, cp.r2_lo) * cs.irho;
    const float dr = cs.drho * cs.irho;
    sd[0] -= dr;
    sd[3] -= dr;
    if constexpr (D == 3) sd[5] -= dr;
    const float iso = __builtin_fmaf(cp.kappa, cs.Teq1 - cs.Ttr1, cs.Ttr1);
#pragma unroll
    for (int k = 0; k < 6; k++) A[k] = beta * sd[k];
    // trace-free part of sigma: subtract T_tr - 1 on the diagonal
    A[0] = __builtin_fmaf(-beta, cs.Ttr1, A[0]) + iso;
    A[3] = __builtin_fmaf(-beta, cs.Ttr1, A[3]) + iso;
    if constexpr (D == 3) A[5] = __builtin_fmaf(-beta, cs.Ttr1, A[5]) + iso;
}

// --------------------------------------------------------------------------
// The collision of one cell: F, E in/out (scaled deviations).
// --------------------------------------------------------------------------

template <class L, bool HAS_G, class R = double>
__device__ __forceinline__ void collide(const Coll &cp, float *F, float *E) {
    constexpr int D = L::D;
    const CellState<D> cs = cell_moments<L, HAS_G>(cp, F, E);
    float A[6];
    lambda_minus_delta<D>(cp, cs, A);
    float ut[3] = {cs.J[0] * cs.irho, cs.J[1] * cs.irho, cs.J[2] * cs.irho};
    const TargetInv<D, R> T = target_inv<D, R>(A, ut, cp.r2, cp.r2_lo);

    const float om = cp.omega;
    const float rho = cs.rho, drho = cs.drho;
    const float gT = cp.hN * (1.0f + cs.Trel1);  // (N_f/2) T_rel
    const float gT1 = cp.hN * cs.Trel1;          // (N_f/2)(T_rel - 1)

    // rest direction
    {
        const float X = float(target_x<R>(target_rest<D, R>(T), rho, drho, cp.wh[0], cp.wl[0]));
        F[0] = __builtin_fmaf(om, X - F[0], F[0]);
        if constexpr (HAS_G) {
            const float gt = __builtin_fmaf(gT, X, mul2(gT1, cp.wh[0], cp.wl[0]));
            E[0] = __builtin_fmaf(om, gt - E[0], E[0]);
        }
    }
    // velocity pairs: relax, and accumulate the post-collision mass and
    // momentum of f per shell for the projection
    float pm = F[0] * cp.isc[0], pJ[3] = {0, 0, 0};
    float m0 = 0, j0 = 0, j1 = 0, j2 = 0;
    static_for<L::NP>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        constexpr int cx = L::P[p].c[0], cy = L::P[p].c[1], cz = L::P[p].c[2];
        constexpr int sh = L::P[p].shell;
        constexpr int a = 2 * p + 1, b = 2 * p + 2;
        if constexpr (first_in_shell<L, p>()) m0 = j0 = j1 = j2 = 0;
        R Em1, O;
        target_pair<D, cx, cy, cz, R>(T, Em1, O);
        const float w = cp.wh[sh], wl = cp.wl[sh];
        const R X = target_x<R>(Em1, rho, drho, w, wl), Y = target_y<R>(O, rho, w, wl);
        const float Ga = float(X + Y), Gb = float(X - Y);
        const float fa = __builtin_fmaf(om, Ga - F[a], F[a]);
        const float fb = __builtin_fmaf(om, Gb - F[b], F[b]);
        F[a] = fa;
        F[b] = fb;
        if constexpr (HAS_G) {
            const float c0 = mul2(gT1, w, wl);
            const float ga = __builtin_fmaf(gT, Ga, c0), gb = __builtin_fmaf(gT, Gb, c0);
            E[a] = __builtin_fmaf(om, ga - E[a], E[a]);
            E[b] = __builtin_fmaf(om, gb - E[b], E[b]);
        }
        const float sp = fa + fb, dp = fa - fb;
        m0 += sp;
        j0 = acc_c<cx>(j0, dp);
        j1 = acc_c<cy>(j1, dp);
        if constexpr (D == 3) j2 = acc_c<cz>(j2, dp);
        if constexpr (last_in_shell<L, p>()) {
            const float is = cp.isc[sh];
            pm = __builtin_fmaf(m0, is, pm);
            pJ[0] = __builtin_fmaf(j0, is, pJ[0]);
            pJ[1] = __builtin_fmaf(j1, is, pJ[1]);
            if constexpr (D == 3) pJ[2] = __builtin_fmaf(j2, is, pJ[2]);
        }
    });
    // projection: f_i += w_i (dM + xi_i . dj), scaled: F_i += wh_i (dM + r^2 c_i . dJ)
    const float dM = drho - pm;
    const float dJ0 = cp.r2 * (cs.J[0] - pJ[0]);
    const float dJ1 = cp.r2 * (cs.J[1] - pJ[1]);
    const float dJ2 = D == 3 ? cp.r2 * (cs.J[2] - pJ[2]) : 0.f;
    F[0] = __builtin_fmaf(cp.wh[0], dM, F[0]);
    static_for<L::NP>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        constexpr int cx = L::P[p].c[0], cy = L::P[p].c[1], cz = L::P[p].c[2];
        constexpr int sh = L::P[p].shell;
        float cj = 0;
        cj = acc_c<cx>(cj, dJ0);
        cj = acc_c<cy>(cj, dJ1);
        if constexpr (D == 3) cj = acc_c<cz>(cj, dJ2);
        const float w = cp.wh[sh];
        F[2 * p + 1] = __builtin_fmaf(w, dM + cj, F[2 * p + 1]);
        F[2 * p + 2] = __builtin_fmaf(w, dM - cj, F[2 * p + 2]);
    });
}

// Equilibrium populations of (drho, u (physical), dT): f = G(rho, u, T delta),
// g = (N_f/2) T G, as scaled deviations.
template <class L, bool HAS_G>
__device__ __forceinline__ void equilibrium(const Coll &cp, float drho, const float *u_phys, float dT, float *F,
                                            float *E) {
    constexpr int D = L::D;
    const float rho = 1.0f + drho;
    float A[6] = {0, 0, 0, 0, 0, 0};
    A[0] = dT;
    A[3] = dT;
    if constexpr (D == 3) A[5] = dT;
    // u = r ut  ->  ut = u / r;  r^2 ut = r u
    const float r = __builtin_sqrtf(cp.r2);
    float ut[3] = {u_phys[0] / r, u_phys[1] / r, D == 3 ? u_phys[2] / r : 0.f};
    const TargetInv<D, double> T = target_inv<D, double>(A, ut, cp.r2, cp.r2_lo);
    const float gT = cp.hN * (1.0f + dT), gT1 = cp.hN * dT;
    const float X0 = float(target_x<double>(target_rest<D, double>(T), rho, drho, cp.wh[0], cp.wl[0]));
    F[0] = X0;
    if constexpr (HAS_G) E[0] = __builtin_fmaf(gT, X0, mul2(gT1, cp.wh[0], cp.wl[0]));
    static_for<L::NP>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        constexpr int cx = L::P[p].c[0], cy = L::P[p].c[1], cz = L::P[p].c[2];
        double Em1, O;
        target_pair<D, cx, cy, cz, double>(T, Em1, O);
        const float w = cp.wh[L::P[p].shell], wl = cp.wl[L::P[p].shell];
        const double X = target_x<double>(Em1, rho, drho, w, wl), Y = target_y<double>(O, rho, w, wl);
        const float Ga = float(X + Y), Gb = float(X - Y);
        F[2 * p + 1] = Ga;
        F[2 * p + 2] = Gb;
        if constexpr (HAS_G) {
            const float c0 = mul2(gT1, w, wl);
            E[2 * p + 1] = __builtin_fmaf(gT, Ga, c0);
            E[2 * p + 2] = __builtin_fmaf(gT, Gb, c0);
        }
    });
}

// Diffusely reflecting walls normal to y (two-copy pull layout).  Rows
// [0, reach) and [ny - reach, ny) are ghost rows outside the gas.  Per wall
// (0 bottom, 1 top), in the library's direction order:
struct WallSet {
    double G[2][MAX_Q];   // G_i(1, u_w, T_w delta): the wall's emission per unit density
    double T[2];          // wall temperatures
    double emit[2];       // sum over gas-bound directions of |c_y| G_i (mass emitted per unit density)
    double rest[2];       // sum over wall-bound directions of |c_y| w_i (rest part of the mass received)
    int reach;
};

// Cache policy code of the step kernels: 0 default; 2 non-temporal loads and
// stores; 3 non-temporal stores with default loads (the reads at x - c_i
// then keep their lines in L2 for the neighbouring work-groups, while the
// stores, read again only in the next step, do not displace them).
constexpr int load_aux(int policy) { return policy == 2 ? 2 : 0; }
constexpr int store_aux(int policy) { return policy == 2 || policy == 3 ? 2 : 0; }

// XCD-aware block order: the eight XCDs take blocks round-robin; give XCD k a
// contiguous run of logical blocks so that neighbouring tiles share its L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb) {
    const uint32_t per = nb >> 3, rem = nb & 7u, xcd = b & 7u, loc = b >> 3;
    return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + loc;
}

}  // namespace esbgk
