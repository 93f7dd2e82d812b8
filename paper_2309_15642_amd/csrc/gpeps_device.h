// Device helpers shared by the forward and adjoint kernels of libgpeps.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gpeps_internal.h"

namespace gpeps {

// ------------------------------------------------------------------ complex helpers

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
template <typename CT> __device__ __forceinline__ CT from_d2(double2 v);
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 v) { return v; }

// Sum over groups of `width` consecutive lanes (width a power of two <= 64).
__device__ __forceinline__ double group_sum(double v, int width) {
  for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// DPP lane permutation of a double (two 32-bit moves).  Only permutations inside a row of 16
// lanes are used, so no source lane is out of range and the moves need no old value.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(b & 0xffffffffull), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over aligned groups of L lanes (L uniform, power of two <= 64): DPP
// quad_perm xor-1 and xor-2, then row_half_mirror (8) and row_mirror (16);
// every lane of a group ends with the group sum.  Wider groups use ds_bpermute.
__device__ __forceinline__ double group_sum_dpp(double v, int L) {
  if (L >= 2) v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  if (L >= 4) v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  if (L >= 8) v += dpp_d<0x141>(v);  // row_half_mirror
  if (L >= 16) v += dpp_d<0x140>(v); // row_mirror
  if (L >= 32) v += __shfl_xor(v, 16, 64);
  if (L >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// group_sum_dpp of two values with the levels of the two sums alternating, so that the
// latency of one sum's step hides behind the other's (each result as group_sum_dpp's, bit for
// bit).
__device__ __forceinline__ void group_sum2_dpp(double& a, double& b, int L) {
  if (L >= 2) { a += dpp_d<0xB1>(a); b += dpp_d<0xB1>(b); }
  if (L >= 4) { a += dpp_d<0x4E>(a); b += dpp_d<0x4E>(b); }
  if (L >= 8) { a += dpp_d<0x141>(a); b += dpp_d<0x141>(b); }
  if (L >= 16) { a += dpp_d<0x140>(a); b += dpp_d<0x140>(b); }
  if (L >= 32) { a += __shfl_xor(a, 16, 64); b += __shfl_xor(b, 16, 64); }
  if (L >= 64) { a += __shfl_xor(a, 32, 64); b += __shfl_xor(b, 32, 64); }
}

// Values of lane l ^ OFF of two 32-bit words (OFF = 4, 8, 16 or 32), with no LDS traffic.  Every
// lane of the wave must be active.  4: row_half_mirror then quad_perm [3,2,1,0]
// (7 - (l ^ 3) = l ^ 4 within 8 lanes); 8: row_ror:8.  16 and 32: v_permlane16_swap(x, y)
// exchanges rows 1, 3 of x with rows 0, 2 of y (rows of 16 lanes), leaving x = [a0 b0 a2 b2],
// y = [a1 b1 a3 b3] for (x, y) = (a, b); the same swap with the operands reversed then leaves
// [a1 a0 a3 a2] and [b1 b0 b3 b2], i.e. both words with their rows exchanged.  v_permlane32_swap
// does the same with halves of 32 lanes.
template <int OFF>
__device__ __forceinline__ void lane_xor2(unsigned& a, unsigned& b) {
  static_assert(OFF == 4 || OFF == 8 || OFF == 16 || OFF == 32, "lane_xor2 offset");
  if constexpr (OFF == 4) {
    a = (unsigned)__builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp((int)a, 0x141, 0xf, 0xf, true), 0x1B, 0xf, 0xf, true);
    b = (unsigned)__builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp((int)b, 0x141, 0xf, 0xf, true), 0x1B, 0xf, 0xf, true);
  } else if constexpr (OFF == 8) {
    a = (unsigned)__builtin_amdgcn_mov_dpp((int)a, 0x128, 0xf, 0xf, true);
    b = (unsigned)__builtin_amdgcn_mov_dpp((int)b, 0x128, 0xf, 0xf, true);
  } else if constexpr (OFF == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    const auto q = __builtin_amdgcn_permlane16_swap(r[1], r[0], false, false);
    a = q[0];
    b = q[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    const auto q = __builtin_amdgcn_permlane32_swap(r[1], r[0], false, false);
    a = q[0];
    b = q[1];
  }
}
// A double with the value of lane l ^ OFF (its two halves form the pair).
template <int OFF>
__device__ __forceinline__ double lane_xor(double v) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  unsigned lo = (unsigned)(bits & 0xffffffffull), hi = (unsigned)(bits >> 32);
  lane_xor2<OFF>(lo, hi);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Values of lane l ^ OFF of two doubles.  The low words of the two are exchanged as one pair
// and the high words as another, so that each result lands whole in a register pair (the
// v_permlane swaps leave their two operands exchanged) and no register copies are needed.
template <int OFF>
__device__ __forceinline__ void lane_xor_pair(double& p, double& q) {
  const unsigned long long bp = (unsigned long long)__double_as_longlong(p);
  const unsigned long long bq = (unsigned long long)__double_as_longlong(q);
  unsigned pl = (unsigned)(bp & 0xffffffffull), ph = (unsigned)(bp >> 32);
  unsigned ql = (unsigned)(bq & 0xffffffffull), qh = (unsigned)(bq >> 32);
  lane_xor2<OFF>(pl, ql);
  lane_xor2<OFF>(ph, qh);
  p = __longlong_as_double((long long)(((unsigned long long)ph << 32) | pl));
  q = __longlong_as_double((long long)(((unsigned long long)qh << 32) | ql));
}

// A complex64 element read or written once: with `stream` the access carries the nontemporal
// hint (no cache allocation), for data far larger than the caches.
__device__ __forceinline__ float2 ld_c64(const float2* p, bool stream) {
  if (!stream) return *p;
  const unsigned long long b = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p));
  return make_float2(__uint_as_float((unsigned)(b & 0xffffffffull)), __uint_as_float((unsigned)(b >> 32)));
}
__device__ __forceinline__ void st_c64(float2* p, float2 v, bool stream) {
  if (!stream) {
    *p = v;
    return;
  }
  const unsigned long long b = (unsigned long long)__float_as_uint(v.x) | ((unsigned long long)__float_as_uint(v.y) << 32);
  __builtin_nontemporal_store(b, reinterpret_cast<unsigned long long*>(p));
}

// Orders LDS traffic between the lanes of one wave: writes before it are seen by reads after it.
// The fences keep the compiler from forwarding a lane's own store or moving reads above writes;
// LDS runs a wave's operations in order, so no hardware wait is needed beyond that.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value of lane `lane` of a double, as a wave-uniform value.
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), lane);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Maximum of an unsigned 32-bit value over the wave, as a wave-uniform value: integer maxima
// with DPP within rows of 16 (quad xor-1, xor-2, half-row and row mirrors), then the four row
// maxima by readlane.  Every lane of the wave must be active.
__device__ __forceinline__ unsigned wave_umax_uniform(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xf, 0xf, true));
  v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xf, 0xf, true));
  v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xf, 0xf, true));
  v = max(v, (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xf, 0xf, true));
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)v, 0), b = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)v, 32), d = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return max(max(a, b), max(c, d));
}

// Maximum over the whole wave as a wave-uniform value: DPP within rows of 16, then readlane.
// Every lane of the wave must be active.
__device__ __forceinline__ double wave_max_uniform(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// Maximum over the whole wave (every lane ends with it): DPP within rows of 16, then ds_bpermute.
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  v = fmax(v, __shfl_xor(v, 16, 64));
  v = fmax(v, __shfl_xor(v, 32, 64));
  return v;
}

// 1/sqrt(x) and 1/x for x > 0: hardware estimate plus two Newton steps (full float64 accuracy).
__device__ __forceinline__ double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * (1.5 - 0.5 * x * r * r);
  r = r * (1.5 - 0.5 * x * r * r);
  return r;
}
// One Newton step only: relative error ~1e-13 (for values that need less than full accuracy).
__device__ __forceinline__ double rsq_nr1(double x) {
  double r = __builtin_amdgcn_rsq(x);
  return r * (1.5 - 0.5 * x * r * r);
}
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * (2.0 - x * r);
  r = r * (2.0 - x * r);
  return r;
}

// RZZ(theta_J) phase g(s,t) = exp(-i theta_J z_s z_t / 2), z_0 = +1, z_1 = -1.
__device__ __forceinline__ double2 gate_phase(const InstParam& ip, int s, int t) {
  const double zz = (s == t) ? 1.0 : -1.0;
  return make_double2(ip.g_c, -ip.g_s * zz);
}

__device__ __forceinline__ void flag_status(int32_t* status, int bits) { atomicOr(status, bits); }

// ------------------------------------------------------------------ site-matrix geometry

// Active geometry of one end of an edge: rows run over the other legs
// (first other leg outer), columns over the edge's own leg.
struct SideGeom {
  int64_t base;  // element offset of physical slice 0
  int64_t pstride;
  int32_t d1, d2;    // active dims of the other legs (1 if absent)
  int32_t s1, s2;    // their strides
  int32_t sq;        // stride of the edge leg
  const double* l1;  // lambdas of the other legs (nullptr if absent)
  const double* l2;
  __device__ __forceinline__ int64_t addr(int p, int m, int k) const {
    const int o1 = m / d2, o2 = m - (m / d2) * d2;
    return base + p * pstride + (int64_t)o1 * s1 + (int64_t)o2 * s2 + (int64_t)k * sq;
  }
  __device__ __forceinline__ double env(int m) const {
    const int o1 = m / d2, o2 = m - (m / d2) * d2;
    double w = 1.0;
    if (l1) w *= l1[o1];
    if (l2) w *= l2[o2];
    return w;
  }
};

__device__ __forceinline__ SideGeom side_geom(const DevState& st, const SideInfo& S) {
  SideGeom g;
  g.base = S.goff;
  g.pstride = S.pstride;
  g.d1 = S.oth[0] >= 0 ? st.chi[S.oth[0]] : 1;
  g.d2 = S.oth[1] >= 0 ? st.chi[S.oth[1]] : 1;
  g.s1 = S.so[0];
  g.s2 = S.so[1];
  g.sq = S.sq;
  g.l1 = S.oth[0] >= 0 ? st.lam + (int64_t)S.oth[0] * st.D : nullptr;
  g.l2 = S.oth[1] >= 0 ? st.lam + (int64_t)S.oth[1] * st.D : nullptr;
  return g;
}

// (slot, end * 2 + slice, row block) of workgroup b of a row-block launch with bps blocks per
// slice of the largest site: through the class's end list when the launch has one (the heavy
// ends first, bps blocks per slice, then the light ones, one block per slice, so that the
// longest workgroups start first), else over the full count x 4 x bps grid.
__device__ __forceinline__ void row_task(const DevState& st, int b, int bps, int& slot, int& sp, int& rb) {
  if (st.rlist) {
    const int nh = 2 * bps * st.rl_heavy;
    if (b < nh) {
      const int h = b / (2 * bps), rem = b - (b / (2 * bps)) * 2 * bps;
      const int en = st.rlist[st.rl_light + h];
      slot = en >> 1;
      sp = ((en & 1) << 1) | (rem >= bps ? 1 : 0);
      rb = rem >= bps ? rem - bps : rem;
    } else {
      const int bb = b - nh;
      const int en = st.rlist[bb >> 1];
      slot = en >> 1;
      sp = ((en & 1) << 1) | (bb & 1);
      rb = 0;
    }
  } else {
    slot = b / (4 * bps);
    const int rem = b - slot * 4 * bps;
    sp = rem / bps;
    rb = rem - sp * bps;
  }
}

// (slot, end, slice) of workgroup b of a launch with one workgroup per (item, end, slice): heavy
// ends first when the launch has the class's end list, else in item order.
__device__ __forceinline__ void end_task(const DevState& st, int b, int& slot, int& side, int& p) {
  if (st.rlist) {
    const int nh = 2 * st.rl_heavy;
    const int en = b < nh ? st.rlist[st.rl_light + (b >> 1)] : st.rlist[(b - nh) >> 1];
    slot = en >> 1;
    side = en & 1;
    p = b & 1;
  } else {
    slot = b >> 2;
    side = (b >> 1) & 1;
    p = b & 1;
  }
}

// Workgroups of a row-block launch over `count` items.
__host__ __device__ inline int row_grid(const DevState& st, int count, int bps) {
  return st.rlist ? 2 * (st.rl_light + st.rl_heavy * bps) : count * 4 * bps;
}

// One 16 x 16 tile of a complex product C[i][j] = sum_k A(i, k) B(k, j), by one wave on
// v_mfma_f64_16x16x4f64 (lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] of each k step
// of 4 and receives C[l / 16 + 4 r][l % 16]), four real products per complex one.  fa(i, k) and
// fb(k, j) return the operands (zero past the matrix); the tile's rows start at i0, its columns
// at j0, K is the inner dimension.  Lane l ends with C[i0 + l / 16 + 4 r][j0 + l % 16] in
// (cr[r], ci[r]).  Every lane of the wave must be active.
typedef double cgemm_d4 __attribute__((ext_vector_type(4)));
template <class FA, class FB>
__device__ __forceinline__ void cgemm_tile(int i0, int j0, int K, FA fa, FB fb, cgemm_d4& cr, cgemm_d4& ci) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  cr = (cgemm_d4){0.0, 0.0, 0.0, 0.0};
  ci = (cgemm_d4){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    double2 a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * u + lk;
      a[u] = fa(i0 + li, k);
      b[u] = fb(k, j0 + li);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (k0 + 4 * u < K) {
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, b[u].x, cr, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[u].y, b[u].y, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, b[u].y, ci, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].y, b[u].x, ci, 0, 0, 0);
      }
    }
  }
}

__device__ __forceinline__ int64_t rbuf_off(const DevState& st, int slot, int side, int p) {
  return (((int64_t)slot * 2 + side) * 2 + p) * st.D * st.D;
}

}  // namespace gpeps
