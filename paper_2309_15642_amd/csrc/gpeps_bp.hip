// Belief propagation (BP) on the norm network <psi|psi> of the graph PEPS, for gfx950.
//
// The simple update's lambda environment is the fixed point of BP on the norm network, and BP
// gauging after each step does not improve on it (Results, discussion of Fig. 3(a)).  These
// kernels run BP on the current state without changing it, which measures how far the
// simple-update gauge is from that fixed point:
//   * site tensors in the symmetric gauge A_v = Gamma_v sqrt(lambda_e) on every leg e;
//   * one message per directed edge, a D x D complex float64 matrix over the ket and bra copies
//     of the bond index (zero outside the active chi_e x chi_e block), starting at
//     identity / chi_e; slot 2 e + d holds the message from end d of edge e into end 1 - d;
//   * k_bp_update: one parallel iteration, one workgroup per directed edge:
//       m[a, a'] = sum_{s, b, b', c, c'} A[s, a, b, c] conj(A[s, a', b', c']) M1[b, b'] M2[c, c']
//     (a on the edge's leg, b and c on the sender's other legs, M1 and M2 the messages into the
//     sender along them), divided by its trace; the largest Frobenius change of a message goes
//     to a residual word;
//   * k_bp_readout: one workgroup per qubit, rho[s, s'] with every leg closed by its incoming
//     message, <Z> = (rho_00 - rho_11) / (rho_00 + rho_11).
// Both evaluate, for each (s, a), Q = M1^T P M2 with P[b, c] = A[s, a, b, c] (two small matrix
// products per wave through LDS), then the dot products of Q with conj(A[s', a', ., .]).  The
// work is a few D^4 multiply-adds per edge, so the kernels are small and latency-bound; they
// keep every value in float64.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "gpeps_device.h"
#include "gpeps_internal.h"

namespace gpeps {

namespace {

constexpr int kBpThreads = 256;
constexpr int kBpWaves = kBpThreads / 64;
// DM: compile-time bound on D (16 or 32) that sizes the LDS arrays; entries of a DM x DM matrix
// per lane.  With complex64 storage and DM = 16 the whole site tensor (<= 64 KB) is staged in
// LDS once per workgroup instead of being re-read from L2 by every dot product.
template <int DM> constexpr int bp_per_lane() { return DM * DM / 64; }
template <typename CT, int DM> constexpr bool bp_stage() { return DM == 16 && sizeof(CT) == 8; }

// Geometry of one site tensor as seen by a BP contraction: leg 0 is `a`, legs 1 and 2 are b, c.
struct BpSite {
  int64_t base;     // element offset of the tensor
  int64_t pstride;  // stride of the physical index
  int32_t st[3];    // element strides of a, b, c (0 when absent)
  int32_t dim[3];   // padded dimensions (D, or 1 when absent)
  int32_t edge[3];  // global edge ids (-1 when absent)
  int32_t in[3];    // message slots into this site along a, b, c (-1 when absent)
};

__device__ __forceinline__ int side_of(const DevState& st, int e, int64_t goff) {
  return st.edges[e].side[0].goff == goff ? 0 : 1;
}

// Loads sqrt(lambda) of the three legs and the incoming messages along b and c into LDS, and
// (for the readout) along a.  Absent legs get a weight of 1 and the 1 x 1 message [[1]].
template <bool LOAD_A_MSG, int DM>
__device__ void bp_load(const DevState& st, const BpSite& g, const double2* msg, double (&sl)[3][DM],
                        double2 (&M)[3][DM][DM + 1]) {
  const int D = st.D;
  const int tid = threadIdx.x;
  for (int i = tid; i < 3 * DM; i += kBpThreads) {
    const int l = i / DM, k = i - l * DM;
    double w = 1.0;
    if (g.edge[l] >= 0 && k < D) w = sqrt(st.lam[(int64_t)g.edge[l] * D + k]);
    sl[l][k] = w;
  }
  for (int l = LOAD_A_MSG ? 0 : 1; l < 3; ++l) {
    if (g.in[l] < 0) {
      if (tid == 0) M[l][0][0] = make_double2(1.0, 0.0);
      continue;
    }
    const double2* src = msg + (int64_t)g.in[l] * D * D;
    for (int i = tid; i < D * D; i += kBpThreads) M[l][i / D][i % D] = src[i];
  }
}

// Q = M1^T P M2 for P[b][c] = A[s, a, b, c] (weighted), left in the lane's registers q[k] for the
// entries j = lane + 64 k (b' = j / dc, c' = j % dc).  Uses the wave's LDS scratch W.  The site
// tensor is read from gam + base (global memory, or its LDS copy with base 0).
template <typename CT, int DM>
__device__ void bp_q(const CT* gam, int64_t base, const BpSite& g, int s, int a, const double (&sl)[3][DM],
                     const double2 (&M)[3][DM][DM + 1], double2 (&W)[DM][DM + 1],
                     double2 (&q)[bp_per_lane<DM>()]) {
  constexpr int PL = bp_per_lane<DM>();
  const int lane = threadIdx.x & 63;
  const int db = g.dim[1], dc = g.dim[2], n = db * dc;
  const int64_t row = base + s * g.pstride + (int64_t)a * g.st[0];
  const double wa = sl[0][a];
  for (int j = lane; j < n; j += 64) {
    const int b = j / dc, c = j - (j / dc) * dc;
    W[b][c] = cscale(to_d2(gam[row + (int64_t)b * g.st[1] + (int64_t)c * g.st[2]]), wa * sl[1][b] * sl[2][c]);
  }
  wave_lds_sync();
  // R = P M2
#pragma unroll
  for (int k = 0; k < PL; ++k) {
    const int j = lane + 64 * k;
    double2 r = make_double2(0.0, 0.0);
    if (j < n) {
      const int b = j / dc, c2 = j - (j / dc) * dc;
      for (int c = 0; c < dc; ++c) r = cadd(r, cmul(W[b][c], M[2][c][c2]));
    }
    q[k] = r;
  }
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < PL; ++k) {
    const int j = lane + 64 * k;
    if (j < n) W[j / dc][j - (j / dc) * dc] = q[k];
  }
  wave_lds_sync();
  // Q = M1^T R
#pragma unroll
  for (int k = 0; k < PL; ++k) {
    const int j = lane + 64 * k;
    double2 r = make_double2(0.0, 0.0);
    if (j < n) {
      const int b2 = j / dc, c2 = j - (j / dc) * dc;
      for (int b = 0; b < db; ++b) r = cadd(r, cmul(M[1][b][b2], W[b][c2]));
    }
    q[k] = r;
  }
  wave_lds_sync();
}

// sum over the wave's entries of q[k] conj(A[s2, a2, b', c']) (weighted): every lane gets the sum.
template <typename CT, int DM>
__device__ double2 bp_dot(const CT* gam, int64_t base, const BpSite& g, int s2, int a2, const double (&sl)[3][DM],
                          const double2 (&q)[bp_per_lane<DM>()]) {
  constexpr int PL = bp_per_lane<DM>();
  const int lane = threadIdx.x & 63;
  const int dc = g.dim[2], n = g.dim[1] * dc;
  const int64_t row = base + s2 * g.pstride + (int64_t)a2 * g.st[0];
  const double wa = sl[0][a2];
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < PL; ++k) {
    const int j = lane + 64 * k;
    if (j < n) {
      const int b = j / dc, c = j - (j / dc) * dc;
      const double2 x = cscale(to_d2(gam[row + (int64_t)b * g.st[1] + (int64_t)c * g.st[2]]), wa * sl[1][b] * sl[2][c]);
      acc = cadd(acc, cmulc(x, q[k]));  // conj(x) q
    }
  }
  acc.x = group_sum_dpp(acc.x, 64);
  acc.y = group_sum_dpp(acc.y, 64);
  return acc;
}

}  // namespace

// Identity / chi_e on the active block of every message of buffer 0; clears the residual word.
__global__ void k_bp_init(DevState st) {
  const int D = st.D;
  const int slot = blockIdx.x;
  const int chi = st.chi[slot >> 1];
  double2* m = st.bp_msg + (int64_t)slot * D * D;
  for (int i = threadIdx.x; i < D * D; i += blockDim.x) {
    const int r = i / D, c = i - (i / D) * D;
    m[i] = make_double2(r == c && r < chi ? 1.0 / chi : 0.0, 0.0);
  }
  if (slot == 0 && threadIdx.x == 0) *st.bp_res = 0ull;
}

// One parallel BP iteration: messages of buffer `src` -> buffer 1 - src; with `record` the
// largest Frobenius change of a message is folded into the residual word.
template <typename CT, int DM>
__global__ __launch_bounds__(kBpThreads) void k_bp_update(DevState st, int src, int record) {
  constexpr bool STAGE = bp_stage<CT, DM>();
  constexpr int PL = bp_per_lane<DM>();
  const int D = st.D;
  const int slot = blockIdx.x, e = slot >> 1, d = slot & 1;
  const SideInfo& S = st.edges[e].side[d];
  BpSite g;
  g.base = S.goff;
  g.pstride = S.pstride;
  g.st[0] = S.sq;
  g.dim[0] = D;
  g.edge[0] = e;
  g.in[0] = -1;
  for (int k = 0; k < 2; ++k) {
    const int f = S.oth[k];
    g.edge[1 + k] = f;
    g.st[1 + k] = f >= 0 ? S.so[k] : 0;
    g.dim[1 + k] = f >= 0 ? D : 1;
    g.in[1 + k] = f >= 0 ? 2 * f + (1 - side_of(st, f, S.goff)) : -1;
  }
  const int64_t nmsg = (int64_t)2 * st.NE * D * D;
  const double2* msg = st.bp_msg + (src ? nmsg : 0);
  double2* out = st.bp_msg + (src ? 0 : nmsg) + (int64_t)slot * D * D;
  const double2* old = msg + (int64_t)slot * D * D;

  __shared__ double sl[3][DM];
  __shared__ double2 M[3][DM][DM + 1];
  __shared__ double2 W[kBpWaves][DM][DM + 1];
  __shared__ double2 R[DM][DM + 1];
  __shared__ double red[kBpThreads];
  __shared__ CT As[STAGE ? 2 * DM * DM * DM : 1];
  bp_load<false, DM>(st, g, msg, sl, M);
  const CT* gam = reinterpret_cast<const CT*>(st.gamma);
  int64_t base = g.base;
  if constexpr (STAGE) {
    // the sender's tensor, 2 D^deg <= 2 DM^3 elements, copied in its own layout
    for (int64_t i = threadIdx.x; i < 2 * g.pstride; i += kBpThreads) As[i] = gam[g.base + i];
    gam = As;
    base = 0;
  }
  __syncthreads();

  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double2 q[PL];
  for (int a = wv; a < D; a += kBpWaves) {
    double2 mine = make_double2(0.0, 0.0);  // R[a][lane] for lane < D
    for (int s = 0; s < 2; ++s) {
      bp_q<CT, DM>(gam, base, g, s, a, sl, M, W[wv], q);
      for (int a2 = 0; a2 < D; ++a2) {
        const double2 v = bp_dot<CT, DM>(gam, base, g, s, a2, sl, q);
        if (lane == a2) mine = cadd(mine, v);
      }
    }
    if (lane < D) R[a][lane] = mine;
  }
  __syncthreads();
  // trace normalisation and residual
  if (threadIdx.x < 64) {
    double t = threadIdx.x < D ? R[threadIdx.x][threadIdx.x].x : 0.0;
    t = group_sum(t, 64);
    if (threadIdx.x == 0) red[0] = t;
  }
  __syncthreads();
  const double tr = red[0];
  const bool good = isfinite(tr) && tr > 0.0;
  const double inv = good ? 1.0 / tr : 0.0;
  __syncthreads();
  double dev = 0.0;
  for (int i = threadIdx.x; i < D * D; i += kBpThreads) {
    const double2 v = cscale(R[i / D][i % D], inv);
    const double2 o = old[i];
    dev += cabs2(csub(v, o));
    out[i] = v;
  }
  red[threadIdx.x] = dev;
  __syncthreads();
  for (int off = kBpThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (!good) flag_status(st.status, kStatusNonFinite);
    const double r = sqrt(red[0]);
    // non-negative doubles order like their bit patterns
    if (record) atomicMax(st.bp_res, (unsigned long long)__double_as_longlong(isfinite(r) ? r : 0.0));
  }
}

// The same iteration for D = 16 on the FP64 matrix cores.  Per physical slice s of the sender's
// weighted tensor A_s[a][b][c] (16 x 16 x 16; absent legs have extent 1: weight 1 at index 0,
// 0 beyond) the message is three complex products:
//   X[a][b][c'] = sum_c A_s[a][b][c] M2[c][c']           (16 tiles, rows b, K = c)
//   Y[a][b'][c'] = sum_b M1[b][b'] X[a][b][c']           (per a, rows b', K = b; in place over X)
//   m[a][a']   += sum_{b',c'} Y[a][b'][c'] conj(A_s[a'][b'][c'])   (one tile, K = 256)
// on v_mfma_f64_16x16x4f64 (lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives
// D[l / 16 + 4 r][l % 16]; a complex product is four real ones).  Wave w owns the rows a = w + 4 i
// of the first two products (no barrier between them) and a quarter of the K range of the third;
// the four partial tiles are added in a fixed order.  Operands of A come straight from the site
// tensor in global memory with the sqrt(lambda) weights applied on load.
template <typename CT>
__global__ __launch_bounds__(kBpThreads) void k_bp_update_mfma(DevState st, int src, int record) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int N = 16;
  const int D = st.D;  // == 16
  const int slot = blockIdx.x, e = slot >> 1, d = slot & 1;
  const SideInfo& S = st.edges[e].side[d];
  BpSite g;
  g.base = S.goff;
  g.pstride = S.pstride;
  g.st[0] = S.sq;
  g.dim[0] = D;
  g.edge[0] = e;
  g.in[0] = -1;
  for (int k = 0; k < 2; ++k) {
    const int f = S.oth[k];
    g.edge[1 + k] = f;
    g.st[1 + k] = f >= 0 ? S.so[k] : 0;
    g.dim[1 + k] = f >= 0 ? D : 1;
    g.in[1 + k] = f >= 0 ? 2 * f + (1 - side_of(st, f, S.goff)) : -1;
  }
  const int64_t nmsg = (int64_t)2 * st.NE * D * D;
  const double2* msg = st.bp_msg + (src ? nmsg : 0);
  double2* out = st.bp_msg + (src ? 0 : nmsg) + (int64_t)slot * D * D;
  const double2* old = msg + (int64_t)slot * D * D;

  __shared__ double sl[3][N];
  __shared__ double2 M[3][N][N + 1];   // M[1] = M1 (into the sender along b), M[2] = M2 (along c)
  __shared__ double2 X[N][N][N + 1];   // X[a][b][c'], then Y[a][b'][c']
  __shared__ double2 part[kBpWaves][4][64];
  __shared__ double2 R[N][N + 1];
  __shared__ double red[kBpThreads];
  const int tid = threadIdx.x;
  for (int i = tid; i < 3 * N; i += kBpThreads) {
    const int l = i / N, k = i - (i / N) * N;
    double w = 0.0;
    if (g.edge[l] >= 0) w = k < D ? sqrt(st.lam[(int64_t)g.edge[l] * D + k]) : 0.0;
    else w = k == 0 ? 1.0 : 0.0;
    sl[l][k] = w;
  }
  for (int l = 1; l < 3; ++l) {
    const double2* srcm = g.in[l] >= 0 ? msg + (int64_t)g.in[l] * D * D : nullptr;
    for (int i = tid; i < N * N; i += kBpThreads) {
      const int r = i / N, c = i - (i / N) * N;
      double2 v = make_double2(0.0, 0.0);
      if (srcm) v = srcm[r * D + c];
      else if (r == 0 && c == 0) v = make_double2(1.0, 0.0);
      M[l][r][c] = v;
    }
  }
  __syncthreads();
  const CT* gam = reinterpret_cast<const CT*>(st.gamma);
  // weighted A_s[a][b][c]; indices of an absent leg above 0 carry weight 0 and read element 0
  auto aval = [&](int s, int a, int b, int c) -> double2 {
    const int ac = a < g.dim[0] ? a : 0, bc = b < g.dim[1] ? b : 0, cc = c < g.dim[2] ? c : 0;
    const double w = sl[0][a] * sl[1][b] * sl[2][c];
    const double2 v = to_d2(gam[g.base + s * g.pstride + (int64_t)ac * g.st[0] + (int64_t)bc * g.st[1] +
                                (int64_t)cc * g.st[2]]);
    return cscale(v, w);
  };
  const int l = tid & 63, wv = tid >> 6, li = l & 15, lk = l >> 4;
  d4 mr = {0.0, 0.0, 0.0, 0.0}, mi = {0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < 2; ++s) {
    for (int a = wv; a < N; a += kBpWaves) {
      // X[a] = A_s[a] M2: rows b (li), K = c
      d4 xr = {0.0, 0.0, 0.0, 0.0}, xi = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int c = 4 * ks + lk;
        const double2 av = aval(s, a, li, c);
        const double2 bv = M[2][c][li];
        xr = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, xr, 0, 0, 0);
        xr = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.y, bv.y, xr, 0, 0, 0);
        xi = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.y, xi, 0, 0, 0);
        xi = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.x, xi, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) X[a][lk + 4 * r][li] = make_double2(xr[r], xi[r]);
      wave_lds_sync();
      // Y[a] = M1^T X[a]: rows b' (li), K = b
      d4 yr = {0.0, 0.0, 0.0, 0.0}, yi = {0.0, 0.0, 0.0, 0.0};
      double2 av4[4], bv4[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int b = 4 * ks + lk;
        av4[ks] = M[1][b][li];
        bv4[ks] = X[a][b][li];
      }
      wave_lds_sync();
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        yr = __builtin_amdgcn_mfma_f64_16x16x4f64(av4[ks].x, bv4[ks].x, yr, 0, 0, 0);
        yr = __builtin_amdgcn_mfma_f64_16x16x4f64(-av4[ks].y, bv4[ks].y, yr, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f64_16x16x4f64(av4[ks].x, bv4[ks].y, yi, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f64_16x16x4f64(av4[ks].y, bv4[ks].x, yi, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) X[a][lk + 4 * r][li] = make_double2(yr[r], yi[r]);
    }
    __syncthreads();
    // m[a][a'] += sum_k Y[a][k] conj(A_s[a'][k]), k = 16 b' + c', this wave's 64 values of k
#pragma unroll 4
    for (int ks = 0; ks < 16; ++ks) {
      const int k = 64 * wv + 4 * ks + lk;
      const int bp = k >> 4, cp = k & 15;
      const double2 yv = X[li][bp][cp];
      const double2 cv = cconj(aval(s, li, bp, cp));
      mr = __builtin_amdgcn_mfma_f64_16x16x4f64(yv.x, cv.x, mr, 0, 0, 0);
      mr = __builtin_amdgcn_mfma_f64_16x16x4f64(-yv.y, cv.y, mr, 0, 0, 0);
      mi = __builtin_amdgcn_mfma_f64_16x16x4f64(yv.x, cv.y, mi, 0, 0, 0);
      mi = __builtin_amdgcn_mfma_f64_16x16x4f64(yv.y, cv.x, mi, 0, 0, 0);
    }
    __syncthreads();  // X is overwritten by the next slice
  }
  // partial tiles of the four waves, added in a fixed order: (0 + 1) + (2 + 3)
#pragma unroll
  for (int r = 0; r < 4; ++r) part[wv][r][l] = make_double2(mr[r], mi[r]);
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double2 p0 = part[0][r][l], p1 = part[1][r][l], p2 = part[2][r][l], p3 = part[3][r][l];
      R[lk + 4 * r][li] = cadd(cadd(p0, p1), cadd(p2, p3));
    }
  }
  __syncthreads();
  // trace normalisation and residual (as k_bp_update)
  if (tid < 64) {
    double t = tid < D ? R[tid][tid].x : 0.0;
    t = group_sum(t, 64);
    if (tid == 0) red[0] = t;
  }
  __syncthreads();
  const double tr = red[0];
  const bool good = isfinite(tr) && tr > 0.0;
  const double inv = good ? 1.0 / tr : 0.0;
  __syncthreads();
  double dev = 0.0;
  for (int i = tid; i < D * D; i += kBpThreads) {
    const double2 v = cscale(R[i / D][i % D], inv);
    const double2 o = old[i];
    dev += cabs2(csub(v, o));
    out[i] = v;
  }
  red[tid] = dev;
  __syncthreads();
  for (int off = kBpThreads / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) {
    if (!good) flag_status(st.status, kStatusNonFinite);
    const double r = sqrt(red[0]);
    if (record) atomicMax(st.bp_res, (unsigned long long)__double_as_longlong(isfinite(r) ? r : 0.0));
  }
}

// BP readout of every qubit from the messages of buffer `buf` into st.z.
template <typename CT, int DM>
__global__ __launch_bounds__(kBpThreads) void k_bp_readout(DevState st, int buf) {
  constexpr bool STAGE = bp_stage<CT, DM>();
  constexpr int PL = bp_per_lane<DM>();
  const int D = st.D;
  const int v = blockIdx.x;
  const VertexInfo& V = st.verts[v];
  BpSite g;
  g.base = V.goff;
  int64_t ps = 1;
  for (int l = 0; l < V.deg; ++l) ps *= D;
  g.pstride = ps;
  int64_t stride = ps;
  for (int l = 0; l < 3; ++l) {
    const int f = l < V.deg ? V.leg[l] : -1;
    g.edge[l] = f;
    if (f >= 0) stride /= D;
    g.st[l] = f >= 0 ? (int32_t)stride : 0;
    g.dim[l] = f >= 0 ? D : 1;
    g.in[l] = f >= 0 ? 2 * f + (1 - side_of(st, f, V.goff)) : -1;
  }
  const int64_t nmsg = (int64_t)2 * st.NE * D * D;
  const double2* msg = st.bp_msg + (buf ? nmsg : 0);

  __shared__ double sl[3][DM];
  __shared__ double2 M[3][DM][DM + 1];
  __shared__ double2 W[kBpWaves][DM][DM + 1];
  __shared__ double2 rho[kBpWaves][2][2];
  __shared__ CT As[STAGE ? 2 * DM * DM * DM : 1];
  bp_load<true, DM>(st, g, msg, sl, M);
  const CT* gam = reinterpret_cast<const CT*>(st.gamma);
  int64_t base = g.base;
  if constexpr (STAGE) {
    for (int64_t i = threadIdx.x; i < 2 * g.pstride; i += kBpThreads) As[i] = gam[g.base + i];
    gam = As;
    base = 0;
  }
  __syncthreads();

  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int da = g.dim[0];
  double2 acc[2][2] = {{make_double2(0.0, 0.0), make_double2(0.0, 0.0)},
                       {make_double2(0.0, 0.0), make_double2(0.0, 0.0)}};
  double2 q[PL];
  for (int a = wv; a < da; a += kBpWaves) {
    for (int s = 0; s < 2; ++s) {
      bp_q<CT, DM>(gam, base, g, s, a, sl, M, W[wv], q);
      for (int s2 = 0; s2 < 2; ++s2) {
        // sum_{a'} M0[a][a'] y[s2][a'], y[s2][a'] = <Q, A[s2, a', ., .]>
        double2 t = make_double2(0.0, 0.0);
        for (int a2 = 0; a2 < da; ++a2) t = cadd(t, cmul(M[0][a][a2], bp_dot<CT, DM>(gam, base, g, s2, a2, sl, q)));
        acc[s][s2] = cadd(acc[s][s2], t);
      }
    }
  }
  if (lane == 0) {
    for (int s = 0; s < 2; ++s)
      for (int s2 = 0; s2 < 2; ++s2) rho[wv][s][s2] = acc[s][s2];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r00 = 0.0, r11 = 0.0;
    for (int w = 0; w < kBpWaves; ++w) {
      r00 += rho[w][0][0].x;
      r11 += rho[w][1][1].x;
    }
    const double zv = (r00 - r11) / (r00 + r11);
    if (!isfinite(zv)) flag_status(st.status, kStatusNonFinite);
    st.z[v] = zv;
  }
}

template <typename CT, int DM>
void launch_bp_t(const DevState& st, int iters, hipStream_t stream) {
  const int slots = 2 * st.NE;
  if (slots > 0) {
    hipLaunchKernelGGL(k_bp_init, dim3(slots), dim3(256), 0, stream, st);
    for (int it = 0; it < iters; ++it) {
      if (DM == 16 && st.D == 16)
        hipLaunchKernelGGL((k_bp_update_mfma<CT>), dim3(slots), dim3(kBpThreads), 0, stream, st, it & 1,
                           (int)(it == iters - 1));
      else
        hipLaunchKernelGGL((k_bp_update<CT, DM>), dim3(slots), dim3(kBpThreads), 0, stream, st, it & 1,
                           (int)(it == iters - 1));
    }
  }
  if (st.NV > 0) hipLaunchKernelGGL((k_bp_readout<CT, DM>), dim3(st.NV), dim3(kBpThreads), 0, stream, st, iters & 1);
}

// ------------------------------------------------------------------ device-resident BP scratch
//
// The messages and the residual word of gpeps_bp_expect_z_noalloc live in this array instead of
// the caller's workspace, for callers that cannot allocate.  Every GPU the library runs on holds
// its own copy until the process ends; host code never uses the name itself (a host-side stand-in)
// but the device address returned by hipGetSymbolAddress, recorded once per device.
static __device__ __align__(256) unsigned char scratch[kBpScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device, looked up on the first call for that
// device.  Returns the lookup's status (kept per device) and writes the address to *ptr.
hipError_t bp_scratch_address(void** ptr) {
  *ptr = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void* p = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? p : nullptr;
    g_scratch_done[dev] = true;
  }
  *ptr = g_scratch_ptr[dev];
  return g_scratch_err[dev];
}

hipError_t launch_bp(bool c128, const DevState& st, int iters, hipStream_t stream) {
  if (st.D > kMaxD) return hipErrorInvalidValue;
  if (st.D <= 16) {
    if (c128) launch_bp_t<double2, 16>(st, iters, stream);
    else launch_bp_t<float2, 16>(st, iters, stream);
  } else {
    if (c128) launch_bp_t<double2, 32>(st, iters, stream);
    else launch_bp_t<float2, 32>(st, iters, stream);
  }
  return hipGetLastError();
}

}  // namespace gpeps
