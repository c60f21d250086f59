// Device helpers shared by every kernel of libmppi: the counter-based noise source,
// fast FP32 transcendentals and wave64 reductions.  gfx950 only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mppi {

constexpr int kBlock = 256;       // threads per block in every kernel (4 wave64s)
constexpr int kWave = 64;

// ---------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11, Section 4).  Ten rounds; each
// round forms the two 32x32->64 products of counter words 0 and 2 with the round
// multipliers, XORs their high halves into the other two words together with the
// key, and permutes; the key advances by the two Weyl increments between rounds.
// Integer work only: one v_mad_u64_u32 per product and one v_bitop3_b32 per three-way
// XOR on the VALU; the key schedule is uniform (scalar unit).
// ---------------------------------------------------------------------------------
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 32 x 32 -> 64-bit product as one v_mad_u64_u32 (a mul_lo / mul_hi pair otherwise)
    const uint64_t p0 = (uint64_t)c.x * kPhiloxM0;
    const uint64_t p1 = (uint64_t)c.z * kPhiloxM1;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    // each three-way XOR as one v_bitop3_b32 (truth table 0x96: the parity of the inputs)
    c = make_uint4(__builtin_amdgcn_bitop3_b32(hi1, c.y, k0, 0x96), lo1,
                   __builtin_amdgcn_bitop3_b32(hi0, c.w, k1, 0x96), lo0);
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return c;
}

// Uniform in (0, 1]: the top 24 bits plus one, times 2^-24 -- exact in FP32 (the 24-bit
// integer converts exactly and n 2^-24 + 2^-24 is representable, so the FMA rounds nothing).
__device__ __forceinline__ float uniform01(uint32_t x) {
  return fmaf((float)(x >> 8), 0x1p-24f, 0x1p-24f);
}

// Box-Muller (1958) on one pair: r = sqrt(-2 ln ua), angle 2 pi ub.  v_log_f32 is log2,
// v_sin_f32 / v_cos_f32 take the angle in revolutions, so no range reduction is needed.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float &e0, float &e1) {
  const float ua = uniform01(a);
  const float ub = uniform01(b);
  const float r = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(ua));
  e0 = r * __builtin_amdgcn_cosf(ub);
  e1 = r * __builtin_amdgcn_sinf(ub);
}

// Four standard normals with flat indices 4g .. 4g+3 of sample k at iteration `it`
// (flat index of control j at step i is i*m + j).
__device__ __forceinline__ void normals4(uint32_t g, uint32_t k, uint64_t it, uint32_t key0, uint32_t key1,
                                         float e[4]) {
  const uint4 r = philox4x32_10(make_uint4(g, k, (uint32_t)it, (uint32_t)(it >> 32)), key0, key1);
  box_muller(r.x, r.y, e[0], e[1]);
  box_muller(r.z, r.w, e[2], e[3]);
}

// ---------------------------------------------------------------------------------
// FP32 trigonometry for the dynamics: reduce to revolutions in [-1/2, 1/2] and use the
// hardware sin/cos.  Absolute error ~1e-6 for moderate arguments.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ float rev(float x) {
  constexpr float kInv2Pi = 0.159154943091895335769f;
  return fmaf(x, kInv2Pi, -__builtin_rintf(x * kInv2Pi));   // the fraction from the unrounded product
}
__device__ __forceinline__ float fsin(float x) { return __builtin_amdgcn_sinf(rev(x)); }
__device__ __forceinline__ float fcos(float x) { return __builtin_amdgcn_cosf(rev(x)); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ double fsin(double x) { return sin(x); }
__device__ __forceinline__ double fcos(double x) { return cos(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }

// sin and cos of one angle: one shared reduction (FP32: the revolution; FP64: sincos).
__device__ __forceinline__ void fsincos(float x, float &s, float &c) {
  const float r = rev(x);
  s = __builtin_amdgcn_sinf(r);
  c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ void fsincos(double x, double &s, double &c) { sincos(x, &s, &c); }

// ---------------------------------------------------------------------------------
// Lane groups of a wave: broadcast lane J of each aligned group of G lanes to the group
// (DPP quad_perm for 4, DPP row_newbcast for a 16-lane row, ds_swizzle in bit-mask
// mode for a half wave of 32: source lane (lane & 0) | J within each 32-lane half).
// ---------------------------------------------------------------------------------
template <int J>
__device__ __forceinline__ float quad_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), J * 0x55, 0xF, 0xF, false));
}
template <int G, int J>
__device__ __forceinline__ float group_bcast(float v) {
  if constexpr (G == 4) {
    return quad_bcast<J>(v);
  } else if constexpr (G == 16) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + J, 0xF, 0xF, false));  // row_newbcast:J
  } else {
    static_assert(G == 32, "lane groups of 4, 16 or 32");
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), J << 5));  // and 0, or J, xor 0
  }
}

// Prefix sums over each aligned group of G lanes (G = 4, 16 or 32; lj = lane % G), in a
// fixed tree order.  Inclusive: DPP row shifts by 1, 2, 4, 8 (lanes with no source add
// 0); groups of 4 mask the shifts that would cross a quad; groups of 32 then add the
// first row's total (its lane 15, DPP row_bcast:15) into the second row.  Exclusive: the
// inclusive sum of the lane before (0 in the group's first lane; across the row boundary
// of a 32-lane group by a whole-wave shift).
template <int Ctrl>
__device__ __forceinline__ float dpp_or_zero(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), Ctrl, 0xF, 0xF, false));
}
template <int G>
__device__ __forceinline__ float group_scan_incl(float v, int lj) {
  if constexpr (G >= 16) {
    static_assert(G == 16 || G == 32, "lane groups of 4, 16 or 32");
    v += dpp_or_zero<0x111>(v);                    // row_shr:1
    v += dpp_or_zero<0x112>(v);                    // row_shr:2
    v += dpp_or_zero<0x114>(v);                    // row_shr:4
    v += dpp_or_zero<0x118>(v);                    // row_shr:8
    if constexpr (G == 32)                         // rows 1 and 3 add lane 15 of rows 0 and 2
      v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));
  } else {
    static_assert(G == 4, "lane groups of 4, 16 or 32");
    const float t1 = dpp_or_zero<0x111>(v);
    v += lj >= 1 ? t1 : 0.f;
    const float t2 = dpp_or_zero<0x112>(v);
    v += lj >= 2 ? t2 : 0.f;
  }
  return v;
}
template <int G>
__device__ __forceinline__ float group_excl_of_incl(float incl, int lj) {
  if constexpr (G == 32) {
    const float t = dpp_or_zero<0x138>(incl);      // wave_shr:1
    return lj >= 1 ? t : 0.f;
  } else {
    const float t = dpp_or_zero<0x111>(incl);      // row_shr:1
    if constexpr (G == 16) return t;
    else return lj >= 1 ? t : 0.f;
  }
}

// FP64 forms of the group scan, exclusive scan and broadcast (each 32-bit half moved
// with the same DPP or swizzle control; the same tree order as the FP32 forms).
template <int Ctrl, int RowMask = 0xF>
__device__ __forceinline__ double dpp_f64_or_zero(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), Ctrl, RowMask, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), Ctrl, RowMask, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int G>
__device__ __forceinline__ double group_scan_incl_f64(double v, int lj) {
  if constexpr (G >= 16) {
    static_assert(G == 16 || G == 32, "lane groups of 4, 16 or 32");
    v += dpp_f64_or_zero<0x111>(v);                // row_shr:1
    v += dpp_f64_or_zero<0x112>(v);                // row_shr:2
    v += dpp_f64_or_zero<0x114>(v);                // row_shr:4
    v += dpp_f64_or_zero<0x118>(v);                // row_shr:8
    if constexpr (G == 32) v += dpp_f64_or_zero<0x142, 0xA>(v);   // row_bcast:15 into rows 1, 3
  } else {
    static_assert(G == 4, "lane groups of 4, 16 or 32");
    const double t1 = dpp_f64_or_zero<0x111>(v);
    v += lj >= 1 ? t1 : 0.0;
    const double t2 = dpp_f64_or_zero<0x112>(v);
    v += lj >= 2 ? t2 : 0.0;
  }
  return v;
}
template <int G>
__device__ __forceinline__ double group_excl_of_incl_f64(double incl, int lj) {
  if constexpr (G == 32) {
    const double t = dpp_f64_or_zero<0x138>(incl);   // wave_shr:1
    return lj >= 1 ? t : 0.0;
  } else {
    const double t = dpp_f64_or_zero<0x111>(incl);   // row_shr:1
    if constexpr (G == 16) return t;
    else return lj >= 1 ? t : 0.0;
  }
}
template <int G, int J>
__device__ __forceinline__ double group_bcast_f64(double v) {
  return __hiloint2double(__float_as_int(group_bcast<G, J>(__int_as_float(__double2hiint(v)))),
                          __float_as_int(group_bcast<G, J>(__int_as_float(__double2loint(v)))));
}

// Scan of affine maps x -> A x + B over each aligned group of G lanes, composed in lane
// order (a lane's map applies after those of the lanes before it): inclusive result in
// (A, B); lanes with no source take the identity (1, 0).
template <int Ctrl>
__device__ __forceinline__ float dpp_or(float v, float fill) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v), Ctrl, 0xF, 0xF, false));
}
template <int G, int Ctrl, int D>
__device__ __forceinline__ void affine_step(float &A, float &B, int lj) {
  float Ap = dpp_or<Ctrl>(A, 1.f), Bp = dpp_or<Ctrl>(B, 0.f);
  if constexpr (G == 4) {
    if (lj < D) { Ap = 1.f; Bp = 0.f; }            // no crossing into the previous quad
  }
  B = fmaf(A, Bp, B);                              // x -> A (Ap x + Bp) + B
  A = A * Ap;
}
template <int G>
__device__ __forceinline__ void group_affine_scan_incl(float &A, float &B, int lj) {
  affine_step<G, 0x111, 1>(A, B, lj);              // row_shr:1
  affine_step<G, 0x112, 2>(A, B, lj);              // row_shr:2
  if constexpr (G == 16) {
    affine_step<G, 0x114, 4>(A, B, lj);            // row_shr:4
    affine_step<G, 0x118, 8>(A, B, lj);            // row_shr:8
  }
}
// The inclusive map of the lane before (the identity in the group's first lane).
template <int G>
__device__ __forceinline__ void group_affine_excl_of_incl(float &A, float &B, int lj) {
  float Ap = dpp_or<0x111>(A, 1.f), Bp = dpp_or<0x111>(B, 0.f);
  if constexpr (G == 4) {
    if (lj < 1) { Ap = 1.f; Bp = 0.f; }
  }
  A = Ap;
  B = Bp;
}

// Compile-time loop: f(std::integral_constant<int, J>) for J = B .. E-1.
template <int B, int E>
struct StaticFor {
  template <class F>
  __device__ __forceinline__ static void run(F &&f) {
    if constexpr (B < E) {
      f(std::integral_constant<int, B>{});
      StaticFor<B + 1, E>::run(f);
    }
  }
};

// ---------------------------------------------------------------------------------
// Wave64 / block reductions (fixed order: results do not depend on timing).
// ---------------------------------------------------------------------------------
// DPP move of a double (two 32-bit halves); Ctrl is the DPP control word.
template <int Ctrl>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), Ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), Ctrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Wave reductions with every lane active: a DPP butterfly inside each 16-lane row
// (quad_perm swaps, then row rotations by 4 and 8), after which lane 0 of each row holds
// the row's result; the four rows are then combined from lanes 0, 16, 32, 48 in a fixed
// order.  No LDS traffic (a __shfl would go through the LDS crossbar at every step).
template <class Op>
__device__ __forceinline__ double wave_reduce(double v, Op op) {
  v = op(v, dpp_f64<0xB1>(v));                     // quad_perm(1,0,3,2)
  v = op(v, dpp_f64<0x4E>(v));                     // quad_perm(2,3,0,1)
  v = op(v, dpp_f64<0x124>(v));                    // row_ror:4
  v = op(v, dpp_f64<0x128>(v));                    // row_ror:8
  return op(op(readlane_f64(v, 0), readlane_f64(v, 16)), op(readlane_f64(v, 32), readlane_f64(v, 48)));
}
__device__ __forceinline__ double wave_min(double v) {
  return wave_reduce(v, [](double a, double b) { return fmin(a, b); });
}
__device__ __forceinline__ double wave_sum(double v) {
  return wave_reduce(v, [](double a, double b) { return a + b; });
}

// Min over a 256-thread block; every thread gets the result.
__device__ __forceinline__ double block_min(double v, double *scratch4) {
  v = wave_min(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) scratch4[w] = v;
  __syncthreads();
  return fmin(fmin(scratch4[0], scratch4[1]), fmin(scratch4[2], scratch4[3]));
}

// Sum over a 256-thread block in a fixed tree order; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double *scratch4) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) scratch4[w] = v;
  __syncthreads();
  return (scratch4[0] + scratch4[1]) + (scratch4[2] + scratch4[3]);
}

}  // namespace mppi
