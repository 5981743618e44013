// Device helpers shared by the D2Q9 and D3Q19 kernels: periodic index wrap,
// the bulk chemical potential / pressure of the two free energies, and the
// block reduction of the per-tile diagnostics.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_shared.hpp"

namespace lbm {

__device__ __forceinline__ float dev_log(float x) { return logf(x); }
__device__ __forceinline__ double dev_log(double x) { return log(x); }
__device__ __forceinline__ bool dev_finite(float x) { return isfinite(x); }
__device__ __forceinline__ bool dev_finite(double x) { return isfinite(x); }

// Reciprocal of a finite non-zero float64 value: the hardware approximation refined
// by two Newton-Raphson steps r <- r + r (1 - x r), each doubling the correct bits;
// within about 1 ulp, without the scaling and fix-up steps of a correctly rounded
// division (zero or non-finite x give NaN, which the blow-up flags catch).
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Natural logarithm of a float64 argument by range reduction and the atanh series:
// x = 2^e m with m in [sqrt(1/2), sqrt(2)), and log m = 2 atanh(s) with
// s = (m - 1)/(m + 1), summed as 2 s (1 + s^2/3 + s^4/5 + ... + s^22/23)
// (|s| <= 0.1716: truncation below 1e-18 relative); e ln 2 is added with ln 2 split
// into a 29-bit head (exact products with e) and the tail; s takes the reciprocal
// of (2 + f) above.  Within a few ulp of the exact logarithm; zero,
// negative and non-finite arguments give what the C library's log gives.  The
// equation of state only takes logarithms of finite positive densities, so this
// skips the general routine's extra-precision and special-case work (about a
// third of its instructions).
__device__ __forceinline__ double log_pos(double x) {
    constexpr double kLn2Hi = 0x1.62e42ff000000p-1, kLn2Lo = -0x1.718432a1b0e26p-35;
    int e;
    double m = frexp(x, &e);                     // x = m 2^e, m in [1/2, 1)
    if (m < 0.7071067811865476) {
        m += m;
        --e;
    }
    const double f = m - 1.0;                    // exact
    const double s = f * rcp_nr(2.0 + f);
    const double z = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, z, 1.0 / 21.0);
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    const double hs = s + s;
    const double lm = fma(hs * z, p, hs);
    const double de = (double)e;
    const double r = fma(de, kLn2Hi, fma(de, kLn2Lo, lm));
    if (x > 0.0 && x < __builtin_inf()) return r;
    return x == 0.0 ? -__builtin_inf() : (x > 0.0 ? x : __builtin_nan(""));
}

// Reciprocal and logarithm on the step's critical path: in float64 rcp_nr and
// log_pos above; in float32 the hardware 1-ulp instructions.
__device__ __forceinline__ double dev_rcp(double x) { return rcp_nr(x); }
__device__ __forceinline__ float dev_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double dev_logf(double x) { return log_pos(x); }
__device__ __forceinline__ float dev_logf(float x) { return __logf(x); }

// Load / store at a wave-uniform base plus a 32-bit byte offset, the form the
// hardware takes with the base in scalar registers (no 64-bit lane addresses).
// The populations written by a step are not read again within it, so they are
// stored non-temporally: they stream out during the kernel instead of sitting
// dirty in L2 until the end-of-kernel write-back.
template <typename S>
__device__ __forceinline__ S ld_off(const S* base, unsigned idx) {
    return *reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(S));
}
template <typename S>
__device__ __forceinline__ void st_off(S* base, unsigned idx, S v) {
    __builtin_nontemporal_store(v, reinterpret_cast<S*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(S)));
}

// Store at device scope: written through the L2 to the memory side during the
// kernel, so nothing of it is left for the end-of-kernel write-back.  It pays for
// a lattice whose two state buffers stay in the last-level cache between steps
// (the write-back is then a large part of a short step); streaming lattices keep
// the non-temporal stores above.
template <typename S>
__device__ __forceinline__ void st_dev(S* base, unsigned idx, S v) {
    __hip_atomic_store(reinterpret_cast<S*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(S)), v,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Buffer access to one population array.  A descriptor covers the array (base,
// size in bytes); an access adds a per-lane byte offset (vector register) and a
// wave-uniform byte offset (scalar register), so that a pull whose lane offsets
// are fixed over a sweep costs no vector arithmetic.  The hardware returns 0 for
// loads and drops stores beyond the array.
constexpr int kRawBufferDword3 = 0x00020000;   // untyped 32-bit data, gfx9-family descriptor word 3
constexpr int kBufNonTemporal = 2;             // cache policy bits: nt
constexpr int kBufDeviceScope = 16;            // sc1: written through to the device coherence point
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pop_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRawBufferDword3);
}
template <typename S>
__device__ __forceinline__ S buf_ld(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <int AUX>
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, voff, soff, AUX);
}
template <int AUX>
__device__ __forceinline__ void buf_st(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    typedef int v2i __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, v), r, voff, soff, AUX);
}

// Periodic wrap of a coordinate that is at most a few nodes outside [0, n).
// `slow` is set by the host when n is too small for one conditional correction.
__device__ __forceinline__ int wrap(int v, int n, int slow) {
    if (slow) {
        int r = v % n;
        return r < 0 ? r + n : r;
    }
    v += (v < 0) ? n : 0;
    v -= (v >= n) ? n : 0;
    return v;
}

// Bulk part of the chemical potential, mu_EOS = E_f'(rho), and p_EOS = rho E_f' - E_f.
//   vdW (Eq. 30): E_f = rho R T ln[rho/(1 - b rho)] - a rho^2
//   CS          : E_f = rho R T [ln rho + (4h - 3h^2)/(1 - h)^2] - a rho^2,  h = b rho / 4
template <typename T>
struct Eos {
    int kind;
    T a, b, RT;

    __device__ __forceinline__ T mu(T rho) const;

    __device__ __forceinline__ T p(T rho) const {
        if (kind == 0) return rho * RT / (T(1) - b * rho) - a * rho * rho;
        const T h = T(0.25) * b * rho;
        const T iom = T(1) / (T(1) - h);
        return rho * RT * (T(1) + h + h * h - h * h * h) * (iom * iom * iom) - a * rho * rho;
    }
};

template <typename T>
__device__ __forceinline__ T Eos<T>::mu(T rho) const {
    if (kind == 0) {
        const T ibr = dev_rcp(T(1) - b * rho);
        return RT * (dev_logf(rho * ibr) + ibr) - T(2) * a * rho;
    }
    const T h = T(0.25) * b * rho;
    const T iom = dev_rcp(T(1) - h);
    const T iom3 = iom * iom * iom;
    return RT * (dev_logf(rho) + T(1) + h * (T(8) - T(9) * h + T(3) * h * h) * iom3) - T(2) * a * rho;
}

// Chemical potential in the step kernels' LDS.  Float32 kernels keep density and
// chemical potential as deviations from the lattice's reference state, x = rho -
// rho_ref and mu - mu_ref, and evaluate the bulk part mu_EOS(rho_ref + x) - mu_ref
// in float64 from the exact density.  The float32 evaluation's error (about 1e-7:
// rho rounded to float32 at ~8, cancellation between the EOS terms) drives spurious
// velocities ten times above those that the float32 storage itself leaves (measured
// on the 512^2 droplet: 2.9e-6 against 2.5e-7), while the deviation of the result
// is small and rounds to float32 well below 1e-8.  Float64 kernels keep rho and mu
// themselves (rho_ref = 0, no offset).
#ifndef LBM_MU_FLOAT64
#define LBM_MU_FLOAT64 0
#endif
struct MuRef {
    int kind;
    double a, b, RT, rho_ref, mu_off, q0, k0;
    __device__ __forceinline__ MuRef(const LatticeRec& R, bool f32)
        : kind(R.eos), a(R.a), b(R.b), RT(R.RT), rho_ref(R.rho_ref), mu_off(f32 ? R.mu_ref : 0.0), q0(R.dev_q0),
          k0(R.dev_k0) {}
    // bulk chemical potential minus the LDS offset at density rho_ref + x
    template <typename T>
    __device__ __forceinline__ T dmu(const Eos<T>& eos, T x) const {
        if constexpr (sizeof(T) == 4) {
            if constexpr (LBM_MU_FLOAT64) {
                const Eos<double> e{kind, a, b, RT};
                return (T)(e.mu(rho_ref + (double)x) - mu_off);
            } else {
                // float32 in deviation form: with q = 1/(1 - b rho) (vdW) the x-dependent
                // parts are RT [ln(rho q) + b x q q0] - 2 a x; with q = 1/(1 - h), h = b rho/4
                // (CS) they are RT [ln rho + g(h) - g(h0)] - 2 a x, g = 2 q^3 + q^2 - 3, and
                // g(h) - g(h0) = (h - h0) q q0 (2 (q^2 + q q0 + q0^2) + q + q0); k0 holds the rest
                const T rt = (T)RT, bb = (T)b, qq0 = (T)q0, r = (T)rho_ref + x;
                if (kind == 0) {
                    const T q = dev_rcp(dev_rcp(qq0) - bb * x);
                    return (T)k0 + rt * (dev_logf(r * q) + bb * x * q * qq0) - T(2) * (T)a * x;
                }
                const T dh = T(0.25) * bb * x;
                const T q = dev_rcp(dev_rcp(qq0) - dh);
                const T g = dh * q * qq0 * (T(2) * (q * q + q * qq0 + qq0 * qq0) + q + qq0);
                return (T)k0 + rt * (dev_logf(r) + g) - T(2) * (T)a * x;
            }
        } else {
            return eos.mu(x);
        }
    }
};

// Block -> tile mapping that keeps spatially adjacent tiles on one XCD: work
// groups are dealt to the 8 XCDs round-robin, so block b runs on XCD b % 8 and
// is given tile (b % 8) * tiles_per_xcd + b / 8 of the spatially ordered list.
__device__ __forceinline__ int tile_of_block(int b, int tiles_per_xcd) {
    return (b & 7) * tiles_per_xcd + (b >> 3);
}

// Wave reductions without LDS traffic: four DPP butterflies inside each 16-lane
// row (quad permutations [1,0,3,2] and [2,3,0,1], then the half-row and row
// mirrors) leave every lane holding its row's result, and the rows are combined
// from lanes 0, 16, 32 and 48 in that order.  A lane and its partner compute
// op(a, b) and op(b, a), equal for these commutative operations, so the result
// does not depend on the lane.  All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u32(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = dpp_u32<CTRL>((unsigned)u), hi = dpp_u32<CTRL>((unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double lane_f64(double v, int lane) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <typename Op>
__device__ __forceinline__ double wave_reduce(double v, Op op) {
    v = op(v, dpp_f64<0xB1>(v));         // quad_perm [1,0,3,2]
    v = op(v, dpp_f64<0x4E>(v));         // quad_perm [2,3,0,1]
    v = op(v, dpp_f64<0x141>(v));        // row_half_mirror
    v = op(v, dpp_f64<0x140>(v));        // row_mirror
    return op(op(lane_f64(v, 0), lane_f64(v, 16)), op(lane_f64(v, 32), lane_f64(v, 48)));
}
__device__ __forceinline__ double wave_sum(double v) {
    return wave_reduce(v, [](double a, double b) { return a + b; });
}
__device__ __forceinline__ double wave_max(double v) {
    return wave_reduce(v, [](double a, double b) { return fmax(a, b); });
}
__device__ __forceinline__ double wave_min(double v) {
    return wave_reduce(v, [](double a, double b) { return fmin(a, b); });
}
__device__ __forceinline__ unsigned wave_or(unsigned v) {
    v |= dpp_u32<0xB1>(v);
    v |= dpp_u32<0x4E>(v);
    v |= dpp_u32<0x141>(v);
    v |= dpp_u32<0x140>(v);
    return ((unsigned)__builtin_amdgcn_readlane((int)v, 0) | (unsigned)__builtin_amdgcn_readlane((int)v, 16)) |
           ((unsigned)__builtin_amdgcn_readlane((int)v, 32) | (unsigned)__builtin_amdgcn_readlane((int)v, 48));
}

// Per-thread diagnostics accumulator, reduced over the block in a fixed order.
struct DiagAcc {
    double mass = 0, mx = 0, my = 0, mz = 0, umax2 = 0;
    double mumin = 1e300, mumax = -1e300;
    unsigned status = 0;
};

// Every wave puts its reduction in LDS and counts its arrival in uscratch[NW]
// (zero on entry); the wave that arrives last sums the slots in wave order (the
// same order whichever wave that is) and stores the record.  No wave waits at a
// barrier, so none waits for the others' global stores to complete.  Returns the
// tile's status bits in lane 0 of that wave (the value it stored), 0 elsewhere.
template <int NT>
__device__ __forceinline__ unsigned block_reduce_store(const DiagAcc& a, DiagPartial* out, double* scratch,
                                                       unsigned* uscratch) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double v[7] = {wave_sum(a.mass), wave_sum(a.mx), wave_sum(a.my), wave_sum(a.mz),
                   wave_max(a.umax2), wave_min(a.mumin), wave_max(a.mumax)};
    const unsigned st = wave_or(a.status);
    if (lane != 0) return 0u;
    for (int k = 0; k < 7; ++k) scratch[k * NW + w] = v[k];
    uscratch[w] = st;
    // the slots are in LDS before the arrival counts (an LDS-only fence: the
    // wave's global stores stay in flight)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    const unsigned before = __hip_atomic_fetch_add(uscratch + NW, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (before != (unsigned)(NW - 1)) return 0u;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    DiagPartial p;
    p.mass = 0; p.momx = 0; p.momy = 0; p.momz = 0;
    p.umax2 = 0; p.mumin = 1e300; p.mumax = -1e300; p.status = 0; p.pad = 0;
    for (int i = 0; i < NW; ++i) {
        p.mass += scratch[0 * NW + i];
        p.momx += scratch[1 * NW + i];
        p.momy += scratch[2 * NW + i];
        p.momz += scratch[3 * NW + i];
        p.umax2 = fmax(p.umax2, scratch[4 * NW + i]);
        p.mumin = fmin(p.mumin, scratch[5 * NW + i]);
        p.mumax = fmax(p.mumax, scratch[6 * NW + i]);
        p.status |= uscratch[i];
    }
    *out = p;
    return p.status;
}

// BGK update of a pair of opposite velocities e and -e (same weight w):
//   f*_(+-) = (1 - omega) f_(+-) + omega feq_(+-) + (1 - omega/2) (G_(+-) + C),
// with feq_(+-) = U + 4.5 w rho eu^2 +- (3 w rho + k php) eu  (even +- odd part) and
// G_(+-) = w (9 eu eF - 3 u.F) +- 3 w eF  (Eq. 14 split the same way); U holds the
// u-independent part and -1.5 w rho u^2, C is even.  With the relaxation folded
// into per-class coefficients the even and odd parts are
//   E = e0 + eu (e1 eu + e2 eF),  e0 = omega U + om2 (C - 3 w u.F), e1 = 4.5 omega w rho, e2 = 9 om2 w
//   O = o1 eu + o2 eF,            o1 = omega (3 w rho + k php),        o2 = 3 om2 w
template <typename T>
__device__ __forceinline__ void pair_update(T& fp, T& fm, T eu, T eF, T e0, T e1, T e2, T o1, T o2, T om1) {
    const T E = e0 + eu * (e1 * eu + e2 * eF);
    const T O = o1 * eu + o2 * eF;
    fp = om1 * fp + (E + O);
    fm = om1 * fm + (E - O);
}

// Float32 storage keeps each node's mass: the difference between the node's
// incoming mass (the float64 sum of its incoming float32 values, exact) and the
// outgoing populations as they will be stored is spread equally over the NAX axis
// populations (their deviations are small, so the residual rounding is ~1e-10 per
// node; the correction carries no momentum and adds to the second moment's trace
// only).  Without it, per-step changes smaller than half an ulp of the large rest
// deviation (~|rho - rho_ref|) are rounded away in the same direction at every node
// of a slowly relaxing bulk and the lattice drifts in mass (measured: 1e-4 over 5e4
// steps at 512^2).  The collisions update the rest population in increment form,
// f0 + d0 with d0 formed from small quantities only, so that its one large rounding
// is that of the stored value.
template <int Q, typename T>
__device__ __forceinline__ double mass_in(const T (&f)[Q]) {
    double m = 0;
#pragma unroll
    for (int a = 0; a < Q; ++a) m += (double)f[a];
    return m;
}
template <int Q, int NAX, typename T>
__device__ __forceinline__ void keep_mass_on_axes(T (&f)[Q], double m_in) {
    double m = 0;
#pragma unroll
    for (int a = 0; a < Q; ++a) m += (double)f[a];
    const T c = (T)((m_in - m) * (1.0 / NAX));
#pragma unroll
    for (int a = 1; a <= NAX; ++a) f[a] += c;
}

template <typename T>
__device__ __forceinline__ unsigned blowup_bits(T rho, T ux, T uy, T uz, double rho_max) {
    unsigned s = 0;
    if (!(dev_finite(rho) && dev_finite(ux) && dev_finite(uy) && dev_finite(uz))) s |= 1u;
    if (!(rho > T(0))) s |= 2u;
    if ((double)rho >= rho_max) s |= 4u;
    return s;
}

}  // namespace lbm
