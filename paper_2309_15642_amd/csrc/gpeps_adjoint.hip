// Adjoint (reverse sweep) of the graph-PEPS simple update for gfx950.
//
// Loss: L = sum_v c_v <Z_v> of the state after the last recorded Trotter step
// (the mean magnetisation of Fig. 2a when c_v = 1/m).  The forward pass stores the
// state at the start of every step (k_checkpoint).  The reverse sweep restores a
// step's checkpoint, recomputes the step while saving the state before each colour
// class, and then reverses the classes in descending order and the RX layer.
//
// One gate, as the forward kernels compute it (per end sigma and physical slice p):
//   A^(p) = Gamma^(p) * w            (w: product of the other legs' lambdas, per row)
//   R^(p): R^H R = A^H A             (Householder, R only)
//   Theta' = [g(s,t) R_i^(s) diag(lambda) R_j^(t)T]_(s,t) = U S V^H, keep chi
//   T_i^(s) = diag(lambda) sum_t g(s,t) R_j^(t)T V_t S^-1,  T_j^(t) = diag(lambda) sum_s g(s,t) R_i^(s)T conj(U_s) S^-1
//   Gamma'^(p) = Gamma^(p) T^(p),  lambda' = S_chi / ||S_chi||
// and its reverse:
//   k_adj_tbar : T-bar = Gamma^H Gamma'-bar                      (row reduction)
//   k_adj_small: T adjoints -> U-bar, V-bar, S-bar, R-bar, lambda-bar, theta_J-bar;
//                complex SVD backward of Theta' (symmetric gauge term, Lorentzian
//                F_kl = d/(d^2 + 1e-12)/(s_k + s_l), d = s_l - s_k in units of s_0);
//                Theta' backward; QR backward
//   k_adj_rows : Gamma-bar = Gamma'-bar T^H + A-bar * w, and lambda-bar of the other legs
// QR backward.  The function of R above is unchanged by R -> W R for any unitary W
// (the singular values are unchanged and V -> conj(W) V cancels in R^T V), so
// R-bar = 2 R G-bar with G-bar Hermitian, and A-bar = 2 A G-bar = A Y, Y = R^-1 R-bar.
// Y is taken from the regularised normal equations (R^H R + delta I) Y = R^H R-bar
// (Gauss-Jordan in LDS, delta = 1e-13 * max diag(R^H R)), then made Hermitian; no Q and no raw
// R^-1 is needed, so rank-deficient slices (frequent at early steps) stay finite.
// When a slice was not reduced (M <= D_e, R = A) A-bar = R-bar directly.
// Complex adjoints follow x-bar = dL/dRe x + i dL/dIm x.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "gpeps_device.h"
#include "gpeps_internal.h"

namespace gpeps {

constexpr double kEpsF = 1e-12;  // Lorentzian broadening of F (singular-value differences, units of s_0)

__device__ __forceinline__ double2 gate_dphase(const InstParam& ip, int s, int t) {
  // d g / d theta_J = -(i/2) z_s z_t g
  const double2 g = gate_phase(ip, s, t);
  const double zz = (s == t) ? 1.0 : -1.0;
  return make_double2(0.5 * zz * g.y, -0.5 * zz * g.x);
}

// block-wide sum of a double (NT threads, result returned to every thread)
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ checkpoints

// Copy n32 32-bit words from src to dst + (*step_ctr) * slot_words (the history row of this step).
__global__ __launch_bounds__(256) void k_checkpoint(const uint32_t* __restrict__ src, uint32_t* dst,
                                                   int64_t n32, int64_t slot_words, const int32_t* step_ctr,
                                                   int max_steps) {
  const int slot = *step_ctr;
  if (slot >= max_steps) return;
  uint32_t* d = dst + (int64_t)slot * slot_words;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n32; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = src[i];
}

__global__ __launch_bounds__(256) void k_fill_d(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// ------------------------------------------------------------------ magnetisation loss

// Mean <Z> over the qubits of every instance from history row `row` (Fig. 2a's magnetisation):
// one workgroup per instance, fixed summation order.
__global__ __launch_bounds__(256) void k_mean_z(DevState st, int row) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  const int vb = st.inst_vb[k], ve = st.inst_vb[k + 1];
  const double* z = st.hist + (int64_t)row * st.NV;
  double acc = 0.0;
  for (int v = vb + (int)threadIdx.x; v < ve; v += 256) acc += z[v];
  const double tot = block_sum<256>(acc, red);
  if (threadIdx.x == 0) st.mean[k] = ve > vb ? tot / (double)(ve - vb) : 0.0;
}

// Seed of the mean-<Z> loss L = sum_k dldm[k] m_k: dL/d<Z_v> = dldm[k] / n_k for v in instance k.
__global__ __launch_bounds__(256) void k_seed_mean(DevState st) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= st.NV) return;
  const int k = st.verts[v].inst;
  const int n = st.inst_vb[k + 1] - st.inst_vb[k];
  const_cast<double*>(st.dldz)[v] = st.dldm[k] / (double)n;
}

// ------------------------------------------------------------------ readout adjoint (seed)

// z_v = (rho00 - rho11)/(rho00 + rho11), rho_ss = sum_x |Gamma[s,x]|^2 W(x), W = prod_l lambda_l[x_l]^2.
template <typename CT>
__global__ __launch_bounds__(256) void k_adj_readout(DevState st) {
  const int v = blockIdx.x;
  const VertexInfo& V = st.verts[v];
  const int D = st.D;
  __shared__ double lw[kMaxDeg][kMaxD];
  __shared__ double acc[kMaxDeg][kMaxD];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kMaxDeg * D; idx += blockDim.x) {
    const int l = idx / D, k = idx - (idx / D) * D;
    double w = 1.0;
    if (l < V.deg) {
      const double x = st.lam[(int64_t)V.leg[l] * D + k];
      w = x * x;
    }
    lw[l][k] = w;
    acc[l][k] = 0.0;
  }
  __syncthreads();
  int64_t ps = 1;
  for (int l = 0; l < V.deg; ++l) ps *= D;
  const CT* gam = reinterpret_cast<const CT*>(st.gamma) + V.goff;
  double r0 = 0.0, r1 = 0.0;
  for (int64_t i = tid; i < ps; i += blockDim.x) {
    double w = 1.0;
    int64_t rest = i;
    for (int l = V.deg - 1; l >= 0; --l) {
      w *= lw[l][(int)(rest % D)];
      rest /= D;
    }
    r0 += cabs2(to_d2(gam[i])) * w;
    r1 += cabs2(to_d2(gam[i + ps])) * w;
  }
  const double rho0 = block_sum<256>(r0, red);
  const double rho1 = block_sum<256>(r1, red);
  const double c = st.dldz[v];
  const double den = (rho0 + rho1) * (rho0 + rho1);
  const double d0 = c * 2.0 * rho1 / den, d1 = -c * 2.0 * rho0 / den;
  double2* gb = st.gbar + V.goff;
  for (int64_t i = tid; i < ps; i += blockDim.x) {
    double w = 1.0;
    int64_t rest = i;
    for (int l = V.deg - 1; l >= 0; --l) {
      w *= lw[l][(int)(rest % D)];
      rest /= D;
    }
    const double2 a = to_d2(gam[i]), b = to_d2(gam[i + ps]);
    gb[i] = cscale(a, 2.0 * d0 * w);
    gb[i + ps] = cscale(b, 2.0 * d1 * w);
  }
  // dL/dW per leg index: for leg l and index k, the sum over the other legs' indices of
  // (d0 |G0|^2 + d1 |G1|^2) w.  The waves take the (l, k) bins in turn; lane j sums the bin's
  // elements j, j + 64, ... and a DPP wave sum adds the lanes, both in a fixed order, so the
  // gradient is bitwise reproducible.
  {
    const int inner = (int)(ps / D);
    const int lane = tid & 63, wv = tid >> 6;
    for (int bin = wv; bin < V.deg * D; bin += 4) {
      const int l = bin / D, k = bin - (bin / D) * D;
      int sl = 1;  // stride of leg l
      for (int l2 = l + 1; l2 < V.deg; ++l2) sl *= D;
      double sacc = 0.0;
      for (int j = lane; j < inner; j += 64) {
        const int hi = j / sl, lo = j - (j / sl) * sl;  // digits above and below leg l
        const int i = (hi * D + k) * sl + lo;
        double w = 1.0;
        int rest = i;
        for (int l2 = V.deg - 1; l2 >= 0; --l2) {
          w *= lw[l2][rest % D];
          rest /= D;
        }
        sacc += (d0 * cabs2(to_d2(gam[i])) + d1 * cabs2(to_d2(gam[i + ps]))) * w;
      }
      sacc = group_sum_dpp(sacc, 64);
      if (lane == 0) acc[l][k] = sacc;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < V.deg * D; idx += blockDim.x) {
    const int l = idx / D, k = idx - (idx / D) * D;
    const double lam = st.lam[(int64_t)V.leg[l] * D + k];
    if (lam > 0.0 && acc[l][k] != 0.0) atomicAdd(&st.lbar[(int64_t)V.leg[l] * D + k], acc[l][k] * 2.0 / lam);
  }
}

// ------------------------------------------------------------------ RX adjoint

// Gamma' = RX Gamma on the physical index: Gamma-bar <- RX^H Gamma-bar,
// theta_h-bar += Re sum conj(Gamma'-bar) dRX Gamma with dRX = [[-s/2, -i c/2], [-i c/2, -s/2]].
template <typename CT>
__global__ __launch_bounds__(256) void k_adj_rx(DevState st, const void* __restrict__ pre, int chunk_first) {
  __shared__ double red[256];
  const int64_t ch = st.chunks[chunk_first + blockIdx.x];
  const int v = (int)(ch >> 32);
  const int cidx = (int)(ch & 0xffffffff);
  const VertexInfo& V = st.verts[v];
  const InstParam ip = st.inst[V.inst];
  int64_t ps = 1;
  for (int l = 0; l < V.deg; ++l) ps *= st.D;
  const CT* g0 = reinterpret_cast<const CT*>(pre) + V.goff;
  double2* gb = st.gbar + V.goff;
  const int64_t i0 = (int64_t)cidx * 1024;
  const double c = ip.rx_c, s = ip.rx_s;
  double part = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i0 + 1024 && i < ps; i += blockDim.x) {
    const double2 a = to_d2(g0[i]), b = to_d2(g0[i + ps]);
    const double2 ba = gb[i], bb = gb[i + ps];
    // dRX Gamma
    const double2 da = make_double2(-0.5 * s * a.x + 0.5 * c * b.y, -0.5 * s * a.y - 0.5 * c * b.x);
    const double2 db = make_double2(0.5 * c * a.y - 0.5 * s * b.x, -0.5 * c * a.x - 0.5 * s * b.y);
    part += cmulc(ba, da).x + cmulc(bb, db).x;
    // RX^H = [[c, i s], [i s, c]]
    gb[i] = make_double2(c * ba.x - s * bb.y, c * ba.y + s * bb.x);
    gb[i + ps] = make_double2(-s * ba.y + c * bb.x, s * ba.x + c * bb.y);
  }
  const double tot = block_sum<256>(part, red);
  // one workgroup per chunk: the chunk's own accumulator, summed per instance at the end
  if (threadIdx.x == 0) st.gpart[st.NE + chunk_first + blockIdx.x] += tot;
}

// ------------------------------------------------------------------ T-bar = Gamma^H Gamma'-bar

template <typename CT>
__global__ __launch_bounds__(256) void k_adj_tbar(DevState st, const int32_t* __restrict__ items, int first) {
  // T-bar[k][k'] = sum_m conj(Gamma[m][k]) Gamma'-bar[m][k'] on the FP64 matrix cores: with
  // v_mfma_f64_16x16x4f64 lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] and receives
  // D[l / 16 + 4 r][l % 16], so the lane reads Gamma and Gamma'-bar at the same (row 4 s + l / 16,
  // column 16 t + l % 16) and the 16 lanes of a row read 16 consecutive columns.  Each wave sums a
  // quarter of the rows; the partial tiles are added in LDS in a fixed order.
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int NT16 = kMaxD / 16;  // column tiles of each operand
  constexpr int UNR = 4;            // row steps (of 4 rows) per load batch
  const int task = blockIdx.x;
  const int slot = task >> 2, side = (task >> 1) & 1, p = task & 1;
  const int e = items[first + slot];
  const SideInfo& S = st.edges[e].side[side];
  const int D = st.D;
  const SlotMeta meta = st.meta[slot];
  const int de = meta.de_old, chi = meta.chi_new;
  const int d1 = S.oth[0] >= 0 ? st.chi[S.oth[0]] : 1;
  const int d2 = S.oth[1] >= 0 ? st.chi[S.oth[1]] : 1;
  const int M = d1 * d2;
  const CT* gam = reinterpret_cast<const CT*>(st.gamma);
  const int64_t base = S.goff + p * S.pstride;
  const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6, li = l & 15, lk = l >> 4;
  const int ta_n = (de + 15) >> 4, tb_n = (chi + 15) >> 4;
  d4 cr[NT16][NT16], ci[NT16][NT16];
#pragma unroll
  for (int ta = 0; ta < NT16; ++ta)
#pragma unroll
    for (int tb = 0; tb < NT16; ++tb) {
      cr[ta][tb] = (d4){0.0, 0.0, 0.0, 0.0};
      ci[ta][tb] = (d4){0.0, 0.0, 0.0, 0.0};
    }
  const int ksteps = (M + 3) >> 2;
  for (int ks0 = wv; ks0 < ksteps; ks0 += 4 * UNR) {
    double2 ga[UNR][NT16], gb[UNR][NT16];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int m = 4 * (ks0 + 4 * u) + lk;
      const bool mv = m < M;
      const int mc = mv ? m : 0;
      const int o1 = mc / d2, o2 = mc - (mc / d2) * d2;
      const int64_t ro = base + (int64_t)o1 * S.so[0] + (int64_t)o2 * S.so[1];
#pragma unroll
      for (int t = 0; t < NT16; ++t) {
        const int c = 16 * t + li;
        ga[u][t] = (mv && c < de) ? to_d2(gam[ro + (int64_t)c * S.sq]) : make_double2(0.0, 0.0);
        gb[u][t] = (mv && c < chi) ? st.gbar[ro + (int64_t)c * S.sq] : make_double2(0.0, 0.0);
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int ta = 0; ta < NT16; ++ta)
#pragma unroll
        for (int tb = 0; tb < NT16; ++tb) {
          if (ta < ta_n && tb < tb_n) {
            // conj(a) b = (a.x b.x + a.y b.y) + i (a.x b.y - a.y b.x)
            cr[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[u][ta].x, gb[u][tb].x, cr[ta][tb], 0, 0, 0);
            cr[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[u][ta].y, gb[u][tb].y, cr[ta][tb], 0, 0, 0);
            ci[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ga[u][ta].x, gb[u][tb].y, ci[ta][tb], 0, 0, 0);
            ci[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ga[u][ta].y, gb[u][tb].x, ci[ta][tb], 0, 0, 0);
          }
        }
  }
  // partial sums of the four waves, added in a fixed order: (0 + 2) + (1 + 3)
  __shared__ double2 part[2][NT16 * NT16 * 4][64];
  if (wv >= 2) {
#pragma unroll
    for (int ta = 0; ta < NT16; ++ta)
#pragma unroll
      for (int tb = 0; tb < NT16; ++tb)
#pragma unroll
        for (int r = 0; r < 4; ++r) part[wv - 2][(ta * NT16 + tb) * 4 + r][l] = make_double2(cr[ta][tb][r], ci[ta][tb][r]);
  }
  __syncthreads();
  if (wv < 2) {
#pragma unroll
    for (int ta = 0; ta < NT16; ++ta)
#pragma unroll
      for (int tb = 0; tb < NT16; ++tb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double2 q = part[wv][(ta * NT16 + tb) * 4 + r][l];
          cr[ta][tb][r] += q.x;
          ci[ta][tb][r] += q.y;
        }
  }
  __syncthreads();
  if (wv == 1) {
#pragma unroll
    for (int ta = 0; ta < NT16; ++ta)
#pragma unroll
      for (int tb = 0; tb < NT16; ++tb)
#pragma unroll
        for (int r = 0; r < 4; ++r) part[0][(ta * NT16 + tb) * 4 + r][l] = make_double2(cr[ta][tb][r], ci[ta][tb][r]);
  }
  __syncthreads();
  if (wv == 0) {
    double2* TB = st.wsb + (int64_t)slot * adj_scratch(D) + (int64_t)(side * 2 + p) * D * D;
#pragma unroll
    for (int ta = 0; ta < NT16; ++ta)
#pragma unroll
      for (int tb = 0; tb < NT16; ++tb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = 16 * ta + lk + 4 * r, kp = 16 * tb + li;
          if (k < de && kp < chi) {
            const double2 q = part[0][(ta * NT16 + tb) * 4 + r][l];
            TB[k * D + kp] = make_double2(cr[ta][tb][r] + q.x, ci[ta][tb][r] + q.y);
          }
        }
  }
}

// ------------------------------------------------------------------ small-matrix edge adjoint

// One small complex product C (+)= op(A) op(B), row-major, m x n with inner dimension k; op bit 0
// transposes, bit 1 conjugates (0 as is, 1 transpose, 2 conjugate, 3 conjugate transpose).
struct Gemm {
  int m, n, k;
  const double2* A;
  int lda, opA;
  const double2* B;
  int ldb, opB;
  double2* C;
  int ldc;
};

__device__ __forceinline__ int gemm_tiles(const Gemm& g) { return ((g.m + 15) >> 4) * ((g.n + 15) >> 4); }

// 16 x 16 output tile `tile` of g, by one wave, on v_mfma_f64_16x16x4f64 (lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16] and receives D[l / 16 + 4 r][l % 16]), four real products per complex one;
// operands are read straight from memory.
__device__ __forceinline__ void gemm_tile(const Gemm& g, int tile, bool accumulate) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  const int tn = (g.n + 15) >> 4, ks = (g.k + 3) >> 2;
  const int ti = tile / tn, tj = tile - (tile / tn) * tn;
  const int i = 16 * ti + li, j = 16 * tj + li;
  d4 cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
  for (int s0 = 0; s0 < ks; s0 += 4) {
    double2 a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = 4 * (s0 + u) + lk;
      a[u] = make_double2(0.0, 0.0);
      b[u] = make_double2(0.0, 0.0);
      if (i < g.m && kk < g.k) {
        a[u] = (g.opA & 1) ? g.A[kk * g.lda + i] : g.A[i * g.lda + kk];
        if (g.opA & 2) a[u] = cconj(a[u]);
      }
      if (j < g.n && kk < g.k) {
        b[u] = (g.opB & 1) ? g.B[j * g.ldb + kk] : g.B[kk * g.ldb + j];
        if (g.opB & 2) b[u] = cconj(b[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (s0 + u < ks) {
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, b[u].x, cr, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[u].y, b[u].y, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, b[u].y, ci, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].y, b[u].x, ci, 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ii = 16 * ti + lk + 4 * r, jj = 16 * tj + li;
    if (ii < g.m && jj < g.n) {
      const double2 v = make_double2(cr[r], ci[r]);
      g.C[ii * g.ldc + jj] = accumulate ? cadd(g.C[ii * g.ldc + jj], v) : v;
    }
  }
}

// NG mutually independent products: their output tiles are spread over the waves of the block
// together, then one barrier.  The descriptors go through LDS (`gd`, at least NG entries, not
// in use by another batch), so each tile reads its product's descriptor with a uniform index.
template <int NG>
__device__ void bgemm_batch(const Gemm (&gs)[NG], Gemm* gd, bool accumulate) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NG; ++i) gd[i] = gs[i];
  }
  int tot = 0;
#pragma unroll
  for (int i = 0; i < NG; ++i) tot += gemm_tiles(gs[i]);
  __syncthreads();
  for (int tile = (int)(threadIdx.x >> 6); tile < tot; tile += (int)(blockDim.x >> 6)) {
    int i = 0, t = tile;
    while (t >= gemm_tiles(gd[i])) {
      t -= gemm_tiles(gd[i]);
      ++i;
    }
    const Gemm g = gd[i];
    gemm_tile(g, t, accumulate);
  }
  __syncthreads();
}

__device__ void bgemm(int m, int n, int k, const double2* A, int lda, int opA, const double2* B, int ldb, int opB,
                      double2* C, int ldc, bool accumulate) {
  const Gemm g = {m, n, k, A, lda, opA, B, ldb, opB, C, ldc};
  for (int tile = (int)(threadIdx.x >> 6); tile < gemm_tiles(g); tile += (int)(blockDim.x >> 6))
    gemm_tile(g, tile, accumulate);
  __syncthreads();
}

// REC: the forward recovered one singular-vector set as Theta' v / sigma (complex64 path), which
// is accurate only to ~2^-52 s_0 / sigma.  Triplets at that noise level (sigma <= kRecTau s_0) are
// then left out of the F terms and their directions go with the orthogonal complement of the
// retained ones, weighted s_k / (s_k^2 + eps_F s_0^2): the value the F term itself takes for a
// partner of vanishing sigma.  A noise-level triplet thus contributes the same whether it is
// retained or not, and the result does not depend on how the forward resolved them.  Without
// REC (both sets accumulated, complex128) every triplet above 1e-13 s_0 is retained and the
// complement takes 1 / s_k.
template <bool REC>
__global__ __launch_bounds__(256) void k_adj_small(DevState st, const int32_t* __restrict__ items, int first,
                                                   double2* __restrict__ ybuf) {
  __shared__ double red[256];
  __shared__ double Sv[2 * kMaxD], Sb[2 * kMaxD], Lb[kMaxD], lam[kMaxD];
  __shared__ int sh_rp;
  __shared__ double Pt[kMaxD][kMaxD + 1];              // elementwise products, reduced by rows / columns
  __shared__ double2 GZ[4][kMaxD][2 * kMaxD + 1];      // [G | Z] of the four QR backwards (Gauss-Jordan)
  __shared__ Gemm gdesc[8];                            // descriptors of a batch of small products
  const int slot = blockIdx.x;
  const int e = items[first + slot];
  const EdgeInfo& E = st.edges[e];
  const InstParam ip = st.inst[E.inst];
  const int D = st.D, NM = 2 * D;
  const int tid = threadIdx.x;
  const SlotMeta meta = st.meta[slot];
  const int de = meta.de_old, chi = meta.chi_new;
  int r[2], Ms[2];
  for (int sd = 0; sd < 2; ++sd) {
    const SideInfo& S = E.side[sd];
    const int d1 = S.oth[0] >= 0 ? st.chi[S.oth[0]] : 1;
    const int d2 = S.oth[1] >= 0 ? st.chi[S.oth[1]] : 1;
    Ms[sd] = d1 * d2;
    r[sd] = min(Ms[sd], de);
  }
  const int ri = r[0], rj = r[1], m0 = 2 * ri, n0 = 2 * rj;
  const int rr = min(m0, n0);
  const int64_t q = (int64_t)D * D;
  double2* base = st.wsb + (int64_t)slot * adj_scratch(D);
  double2* TB = base;
  double2* Ub = base + 4 * q;
  double2* Vb = base + 8 * q;
  double2* J = base + 12 * q;
  double2* K = base + 16 * q;
  double2* In = base + 20 * q;
  double2* M1 = base + 24 * q;
  double2* Vp = base + 28 * q;
  double2* Thb = base + 32 * q;
  double2* X = base + 36 * q;
  double2* Yc = base + 38 * q;
  double2* Xb = base + 40 * q;
  double2* Ycb = base + 42 * q;
  double2* Rb = base + 44 * q;
  double2* H = base + 12 * q;  // [4][D][D] reuses J after the SVD backward
  const double2* U = st.bU + (int64_t)slot * NM * NM;
  const double2* V = st.bV + (int64_t)slot * NM * NM;
  const double2* Rg = st.rbuf + rbuf_off(st, slot, 0, 0);  // i0, i1, j0, j1 blocks of D*D
  const double2* T64 = st.t64 + rbuf_off(st, slot, 0, 0);
  double2* Yout = ybuf + rbuf_off(st, slot, 0, 0);
  const double* lam_g = st.lam + (int64_t)e * D;
  double* lbar_e = st.lbar + (int64_t)e * D;
  const double2 g[2][2] = {{gate_phase(ip, 0, 0), gate_phase(ip, 0, 1)}, {gate_phase(ip, 1, 0), gate_phase(ip, 1, 1)}};
  const double2 dg[2][2] = {{gate_dphase(ip, 0, 0), gate_dphase(ip, 0, 1)},
                            {gate_dphase(ip, 1, 0), gate_dphase(ip, 1, 1)}};

  for (int k = tid; k < rr; k += blockDim.x) Sv[k] = st.bS[(int64_t)slot * NM + k];
  for (int k = tid; k < kMaxD; k += blockDim.x) lam[k] = k < de ? lam_g[k] : 0.0;
  if (tid == 0) {
    int rp = 0;
    const double s0 = st.bS[(int64_t)slot * NM];
    const double tau = REC ? kRecTau : 1e-13;
    for (int k = 0; k < rr; ++k) rp += st.bS[(int64_t)slot * NM + k] > tau * s0;
    sh_rp = rp > chi ? rp : chi;
  }
  __syncthreads();
  const int rp = sh_rp;
  double thj = 0.0;

  // lambda' = S_chi / ||S_chi||  ->  S-bar;  T terms -> S-bar, lambda-bar
  double nrm2 = 0.0, ls = 0.0;
  for (int k = 0; k < chi; ++k) {
    nrm2 += Sv[k] * Sv[k];
    ls += lbar_e[k] * Sv[k];
  }
  const double nrm = sqrt(nrm2);
  // P[k][k'] = sum_w Re conj(TB_w[k][k']) T64_w[k][k'] in parallel, then its column sums give
  // the T terms of S-bar and its row sums those of lambda-bar
  for (int idx = tid; idx < de * chi; idx += blockDim.x) {
    const int k = idx / chi, kp = idx - (idx / chi) * chi;
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) t += cmulc(TB[w * q + k * D + kp], T64[w * q + k * D + kp]).x;
    Pt[k][kp] = t;
  }
  __syncthreads();
  for (int kp = tid; kp < rr; kp += blockDim.x) {
    double sb = 0.0;
    if (kp < chi) {
      sb = lbar_e[kp] / nrm - Sv[kp] * ls / (nrm2 * nrm);
      double t = 0.0;
      for (int k = 0; k < de; ++k) t += Pt[k][kp];
      sb -= t / Sv[kp];
    }
    Sb[kp] = sb;
  }
  for (int k = tid; k < de; k += blockDim.x) {
    double t = 0.0;
    for (int kp = 0; kp < chi; ++kp) t += Pt[k][kp];
    Lb[k] = t / lam[k];
  }
  // X_t = R_j^(t)T V_t[:, :chi],  Yc_s = R_i^(s)T conj(U_s[:, :chi])
  {
    const Gemm gs[4] = {{de, chi, rj, Rg + 2 * q, D, 1, V, NM, 0, X, D},
                        {de, chi, rj, Rg + 3 * q, D, 1, V + rj * NM, NM, 0, X + q, D},
                        {de, chi, ri, Rg, D, 1, U, NM, 2, Yc, D},
                        {de, chi, ri, Rg + q, D, 1, U + ri * NM, NM, 2, Yc + q, D}};
    bgemm_batch(gs, gdesc, false);
  }
  // theta_J and the adjoints of X, Yc
  for (int idx = tid; idx < de * chi; idx += blockDim.x) {
    const int k = idx / chi, kp = idx - (idx / chi) * chi;
    const double f = lam[k] / Sv[kp];
    for (int t = 0; t < 2; ++t) {
      double2 xb = make_double2(0.0, 0.0), ycb = make_double2(0.0, 0.0);
      for (int s = 0; s < 2; ++s) {
        xb = cadd(xb, cmulc(g[s][t], TB[s * q + k * D + kp]));
        ycb = cadd(ycb, cmulc(g[t][s], TB[(2 + s) * q + k * D + kp]));
      }
      Xb[t * q + k * D + kp] = cscale(xb, f);    // sum_s conj(g(s,t)) lambda_k TB_i^(s) / s_k'
      Ycb[t * q + k * D + kp] = cscale(ycb, f);  // (index t here is s): sum_t conj(g(s,t)) lambda TB_j^(t) / s
    }
    for (int s = 0; s < 2; ++s) {
      double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
      for (int t = 0; t < 2; ++t) {
        a = cadd(a, cmul(dg[s][t], X[t * q + k * D + kp]));
        b = cadd(b, cmul(dg[t][s], Yc[t * q + k * D + kp]));
      }
      thj += f * (cmulc(TB[s * q + k * D + kp], a).x + cmulc(TB[(2 + s) * q + k * D + kp], b).x);
    }
  }
  __syncthreads();
  // R-bar_j^(t) = Xb_t^T... : R-bar_j^(t)[b,k] = sum_k' Xb_t[k,k'] conj(V_t[b,k']);  V-bar_t = conj(R_j^(t)) Xb_t
  {
    const Gemm gs[8] = {{rj, de, chi, V, NM, 2, Xb, D, 1, Rb + 2 * q, D},
                        {rj, chi, de, Rg + 2 * q, D, 2, Xb, D, 0, Vb, NM},
                        {rj, de, chi, V + rj * NM, NM, 2, Xb + q, D, 1, Rb + 3 * q, D},
                        {rj, chi, de, Rg + 3 * q, D, 2, Xb + q, D, 0, Vb + rj * NM, NM},
                        {ri, de, chi, U, NM, 0, Ycb, D, 1, Rb, D},
                        {ri, chi, de, Rg, D, 0, Ycb, D, 2, Ub, NM},
                        {ri, de, chi, U + ri * NM, NM, 0, Ycb + q, D, 1, Rb + q, D},
                        {ri, chi, de, Rg + q, D, 0, Ycb + q, D, 2, Ub + ri * NM, NM}};
    bgemm_batch(gs, gdesc, false);
  }
  // zero the columns chi..rp-1 of U-bar, V-bar
  for (int idx = tid; idx < m0 * (rp - chi); idx += blockDim.x) {
    const int a = idx / (rp - chi), c = chi + idx - (idx / (rp - chi)) * (rp - chi);
    Ub[a * NM + c] = make_double2(0.0, 0.0);
  }
  for (int idx = tid; idx < n0 * (rp - chi); idx += blockDim.x) {
    const int a = idx / (rp - chi), c = chi + idx - (idx / (rp - chi)) * (rp - chi);
    Vb[a * NM + c] = make_double2(0.0, 0.0);
  }
  __syncthreads();

  // ---- complex SVD backward over the rp triplets with s > 1e-13 s_0
  {
    const Gemm gs[2] = {{rp, rp, m0, U, NM, 3, Ub, NM, 0, J, NM}, {rp, rp, n0, V, NM, 3, Vb, NM, 0, K, NM}};
    bgemm_batch(gs, gdesc, false);
  }
  const double s0 = Sv[0];
  for (int idx = tid; idx < rp * rp; idx += blockDim.x) {
    const int k = idx / rp, l = idx - (idx / rp) * rp;
    double2 v;
    if (k == l) {
      const double im = (k < chi) ? 0.5 * (J[k * NM + k].y - K[k * NM + k].y) / Sv[k] : 0.0;
      v = make_double2(Sb[k], im);
    } else {
      const double sk = Sv[k] / s0, sl = Sv[l] / s0;
      const double d = sl - sk, ss = sk + sl;
      const double f = ss > 0.0 ? d / (d * d + kEpsF) / ss / (s0 * s0) : 0.0;
      const double2 aj = csub(J[k * NM + l], cconj(J[l * NM + k]));
      const double2 ak = csub(K[k * NM + l], cconj(K[l * NM + k]));
      v = cadd(cscale(aj, f * Sv[l]), cscale(ak, f * Sv[k]));
    }
    In[k * NM + l] = v;
  }
  __syncthreads();
  // U-bar' = (U-bar - U J) S^-1 and V-bar' = (V-bar - V K) S^-1 on the kept columns
  {
    const Gemm gs[2] = {{m0, rp, rp, U, NM, 0, J, NM, 0, M1, NM}, {n0, rp, rp, V, NM, 0, K, NM, 0, Vp, NM}};
    bgemm_batch(gs, gdesc, false);
  }
  // weight of the orthogonal complement of the retained triplets (see REC above)
  auto cw = [&](int l) { return REC ? Sv[l] / (Sv[l] * Sv[l] + kEpsF * s0 * s0) : 1.0 / Sv[l]; };
  for (int idx = tid; idx < m0 * rp; idx += blockDim.x) {
    const int a = idx / rp, l = idx - (idx / rp) * rp;
    M1[a * NM + l] = l < chi ? cscale(csub(Ub[a * NM + l], M1[a * NM + l]), cw(l)) : make_double2(0.0, 0.0);
  }
  for (int idx = tid; idx < n0 * rp; idx += blockDim.x) {
    const int a = idx / rp, l = idx - (idx / rp) * rp;
    Vp[a * NM + l] = l < chi ? cscale(csub(Vb[a * NM + l], Vp[a * NM + l]), cw(l)) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  // M1 += U In ;  Theta'-bar = M1 V^H + U Vp^H
  bgemm(m0, rp, rp, U, NM, 0, In, NM, 0, M1, NM, true);
  bgemm(m0, n0, rp, M1, NM, 0, V, NM, 3, Thb, NM, false);
  bgemm(m0, n0, rp, U, NM, 0, Vp, NM, 3, Thb, NM, true);

  // ---- Theta' backward: H_st = Thb_st conj(R_j^(t))  [ri x de]
  {
    const Gemm gs[4] = {{ri, de, rj, Thb, NM, 0, Rg + 2 * q, D, 2, H, D},
                        {ri, de, rj, Thb + rj, NM, 0, Rg + 3 * q, D, 2, H + q, D},
                        {ri, de, rj, Thb + ri * NM, NM, 0, Rg + 2 * q, D, 2, H + 2 * q, D},
                        {ri, de, rj, Thb + ri * NM + rj, NM, 0, Rg + 3 * q, D, 2, H + 3 * q, D}};
    bgemm_batch(gs, gdesc, false);
  }
  for (int idx = tid; idx < ri * de; idx += blockDim.x) {
    const int a = idx / de, k = idx - (idx / de) * de;
    double lt = 0.0;  // this (a, k)'s share of lambda-bar_k
    for (int s = 0; s < 2; ++s) {
      double2 acc = make_double2(0.0, 0.0);
      const double2 rik = Rg[s * q + a * D + k];
      for (int t = 0; t < 2; ++t) {
        const double2 h = H[(s * 2 + t) * q + a * D + k];
        acc = cadd(acc, cmulc(g[s][t], h));
        thj += lam[k] * cmulc(h, cmul(dg[s][t], rik)).x;
        lt += cmulc(h, cmul(g[s][t], rik)).x;
      }
      Rb[s * q + a * D + k] = cadd(Rb[s * q + a * D + k], cscale(acc, lam[k]));
    }
    Pt[a][k] = lt;
  }
  __syncthreads();
  for (int k = tid; k < de; k += blockDim.x) {
    double t = 0.0;
    for (int a = 0; a < ri; ++a) t += Pt[a][k];
    Lb[k] += t;
  }
  __syncthreads();
  // R-bar_j^(t)[b,k] += lambda_k sum_s conj(g(s,t)) P_st[b,k], P_st = Thb_st^T conj(R_i^(s)) [rj x de]
  // (P_st in the H region, which the loops above have finished with)
  {
    const Gemm gs[4] = {{rj, de, ri, Thb, NM, 1, Rg, D, 2, H, D},
                        {rj, de, ri, Thb + rj, NM, 1, Rg, D, 2, H + q, D},
                        {rj, de, ri, Thb + ri * NM, NM, 1, Rg + q, D, 2, H + 2 * q, D},
                        {rj, de, ri, Thb + ri * NM + rj, NM, 1, Rg + q, D, 2, H + 3 * q, D}};
    bgemm_batch(gs, gdesc, false);
  }
  for (int idx = tid; idx < rj * de; idx += blockDim.x) {
    const int b = idx / de, k = idx - (idx / de) * de;
    for (int t = 0; t < 2; ++t) {
      double2 acc = make_double2(0.0, 0.0);
      for (int s = 0; s < 2; ++s) acc = cadd(acc, cmulc(g[s][t], H[(s * 2 + t) * q + b * D + k]));
      Rb[(2 + t) * q + b * D + k] = cadd(Rb[(2 + t) * q + b * D + k], cscale(acc, lam[k]));
    }
  }
  __syncthreads();

  // ---- QR backward of the four (end, slice) blocks, solved together.  A block that was not
  // reduced (M <= D_e, R = A) has A-bar = R-bar.  For the others G = R^H R and Z = R^H R-bar
  // (one batch of products; G in the H region, finished with above), then
  // Y = (G + delta I)^-1 Z by Gauss-Jordan elimination of [G + delta I | Z] in LDS (Hermitian
  // positive definite: no pivoting), one wave per block and one lane per column, so the four
  // run side by side with no workgroup barrier.
  bool redw[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) redw[w] = Ms[w >> 1] > de;
  for (int w = 0; w < 4; ++w) {
    if (redw[w]) continue;
    const int rows = (w >> 1) ? rj : ri;
    for (int idx = tid; idx < rows * de; idx += blockDim.x) {
      const int a = idx / de, k = idx - (idx / de) * de;
      Yout[w * q + a * D + k] = Rb[w * q + a * D + k];
    }
    if (tid == 0) st.ymode[slot * 4 + w] = 1;
  }
  {
    const int n0r = redw[0] ? de : 0, n1r = redw[1] ? de : 0, n2r = redw[2] ? de : 0, n3r = redw[3] ? de : 0;
    const Gemm gs[8] = {{n0r, de, ri, Rg, D, 3, Rg, D, 0, H, D},
                        {n0r, de, ri, Rg, D, 3, Rb, D, 0, Yout, D},
                        {n1r, de, ri, Rg + q, D, 3, Rg + q, D, 0, H + q, D},
                        {n1r, de, ri, Rg + q, D, 3, Rb + q, D, 0, Yout + q, D},
                        {n2r, de, rj, Rg + 2 * q, D, 3, Rg + 2 * q, D, 0, H + 2 * q, D},
                        {n2r, de, rj, Rg + 2 * q, D, 3, Rb + 2 * q, D, 0, Yout + 2 * q, D},
                        {n3r, de, rj, Rg + 3 * q, D, 3, Rg + 3 * q, D, 0, H + 3 * q, D},
                        {n3r, de, rj, Rg + 3 * q, D, 3, Rb + 3 * q, D, 0, Yout + 3 * q, D}};
    bgemm_batch(gs, gdesc, false);
  }
  {
    // wave w solves system w; lane c owns column c of [G | Z] (G: c < de, Z: kMaxD <= c < kMaxD + de)
    const int wq = tid >> 6, lc = tid & 63;
    if (wq < 4 && redw[wq]) {
      const bool gcol = lc < de, zcol = lc >= kMaxD && lc < kMaxD + de;
      for (int a = 0; a < de; ++a) {
        if (gcol) GZ[wq][a][lc] = H[wq * q + a * D + lc];
        if (zcol) GZ[wq][a][lc] = Yout[wq * q + a * D + lc - kMaxD];
      }
      wave_lds_sync();
      double dmax = gcol ? GZ[wq][lc][lc].x : 0.0;
      dmax = wave_max(dmax);
      if (gcol) GZ[wq][lc][lc].x += 1e-13 * (dmax > 0.0 ? dmax : 1.0);
      wave_lds_sync();
      for (int p = 0; p < de; ++p) {
        // scale row p (columns > p of G and all of Z) by 1 / G[p][p] (real: Hermitian), then
        // eliminate column p from the other rows; column p itself is not written in this step
        const double ip = 1.0 / GZ[wq][p][p].x;
        const bool act = (lc > p && lc < de) || zcol;
        if (act) {
          const double2 rpc = cscale(GZ[wq][p][lc], ip);
          GZ[wq][p][lc] = rpc;
          for (int a = 0; a < de; ++a)
            if (a != p) GZ[wq][a][lc] = csub(GZ[wq][a][lc], cmul(GZ[wq][a][p], rpc));
        }
        wave_lds_sync();
      }
      // Hermitian part of Y
      if (zcol) {
        const int b = lc - kMaxD;
        for (int a = 0; a < de; ++a) {
          const double2 x = GZ[wq][a][kMaxD + b], y = GZ[wq][b][kMaxD + a];
          double2 h = cscale(cadd(x, cconj(y)), 0.5);
          if (a == b) h.y = 0.0;
          Yout[wq * q + a * D + b] = h;
        }
      }
      if (lc == 0) st.ymode[slot * 4 + wq] = 0;
    }
  }
  __syncthreads();

  // ---- pre-gate lambda_e adjoint and dL/dtheta_J
  for (int k = tid; k < D; k += blockDim.x) lbar_e[k] = k < de ? Lb[k] : 0.0;
  const double tot = block_sum<256>(thj, red);
  // one item per edge in a launch: the edge's own accumulator, summed per instance at the end
  if (tid == 0) st.gpart[e] += tot;
}

// ------------------------------------------------------------------ Gamma-bar rows

template <typename CT>
__global__ __launch_bounds__(256) void k_adj_rows(DevState st, const int32_t* __restrict__ items, int first,
                                                  int blocks_per_slice, const double2* __restrict__ ybuf) {
  int slot, sp, rb;
  row_task(st, blockIdx.x, blocks_per_slice, slot, sp, rb);
  const int side = sp >> 1, p = sp & 1;
  const int e = items[first + slot];
  const SideInfo& S = st.edges[e].side[side];
  const int D = st.D;
  const int d1 = S.oth[0] >= 0 ? st.chi[S.oth[0]] : 1;
  const int d2 = S.oth[1] >= 0 ? st.chi[S.oth[1]] : 1;
  const int M = d1 * d2;
  const int row0 = rb * kRowBlock;
  if (row0 >= M) return;
  const int rows = min(kRowBlock, M - row0);
  const SlotMeta meta = st.meta[slot];
  const int de = meta.de_old, chi = meta.chi_new;
  const int ncol = max(de, chi);
  const int mode = st.ymode[slot * 4 + sp];
  // LDS sized by D (dynamic): T [de x chi], Y [de x de] (mode 0), Gamma and Gamma'-bar rows
  extern __shared__ double2 rows_lds[];
  const int DS = D + 1;
  double2* const Ts = rows_lds;
  double2* const Ys = Ts + D * DS;
  double2* const Gs = Ys + D * DS;
  double2* const Bs = Gs + kRowBlock * DS;
  __shared__ double wl[kRowBlock];
  const double* l1 = S.oth[0] >= 0 ? st.lam + (int64_t)S.oth[0] * D : nullptr;
  const double* l2 = S.oth[1] >= 0 ? st.lam + (int64_t)S.oth[1] * D : nullptr;
  const double2* T = st.t64 + rbuf_off(st, slot, side, p);
  const double2* Y = ybuf + rbuf_off(st, slot, side, p);
  const CT* gam = reinterpret_cast<const CT*>(st.gamma);
  const int64_t base = S.goff + p * S.pstride;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < de * chi; idx += blockDim.x) {
    const int k = idx / chi, kp = idx - (idx / chi) * chi;
    Ts[(k) * DS + kp] = T[k * D + kp];
  }
  if (mode == 0) {
    for (int idx = tid; idx < de * de; idx += blockDim.x) {
      const int k = idx / de, l = idx - (idx / de) * de;
      Ys[(k) * DS + l] = Y[k * D + l];
    }
  }
  for (int idx = tid; idx < rows; idx += blockDim.x) {
    const int m = row0 + idx, o1 = m / d2, o2 = m - (m / d2) * d2;
    double w = 1.0;
    if (l1) w *= l1[o1];
    if (l2) w *= l2[o2];
    wl[idx] = w;
  }
  for (int idx = tid; idx < rows * de; idx += blockDim.x) {
    const int rr = idx / de, k = idx - (idx / de) * de;
    const int m = row0 + rr, o1 = m / d2, o2 = m - (m / d2) * d2;
    Gs[(rr) * DS + k] = to_d2(gam[base + (int64_t)o1 * S.so[0] + (int64_t)o2 * S.so[1] + (int64_t)k * S.sq]);
  }
  for (int idx = tid; idx < rows * chi; idx += blockDim.x) {
    const int rr = idx / chi, k = idx - (idx / chi) * chi;
    const int m = row0 + rr, o1 = m / d2, o2 = m - (m / d2) * d2;
    Bs[(rr) * DS + k] = st.gbar[base + (int64_t)o1 * S.so[0] + (int64_t)o2 * S.so[1] + (int64_t)k * S.sq];
  }
  __syncthreads();
  // new Gamma-bar and A-bar per (row, column), w-bar per row: thread t takes row t / 4 of the
  // block and columns t % 4 + 4 j, so its four threads sum a row's w-bar with two DPP steps
  static_assert(kRowBlock * 4 == 256, "one row per four threads");
  __shared__ double wb[kRowBlock];
  {
    const int rr = tid >> 2, kq = tid & 3;
    double wsum = 0.0;
    if (rr < rows) {
      const int m = row0 + rr, o1 = m / d2, o2 = m - (m / d2) * d2;
      const int64_t ro = base + (int64_t)o1 * S.so[0] + (int64_t)o2 * S.so[1];
      for (int k = kq; k < ncol; k += 4) {
        double2 out = make_double2(0.0, 0.0);
        if (k < de) {
          for (int kp = 0; kp < chi; ++kp) out = cadd(out, cmul(Bs[(rr) * DS + kp], cconj(Ts[(k) * DS + kp])));
          double2 abar;
          if (mode == 0) {
            double2 gy = make_double2(0.0, 0.0);
            for (int l = 0; l < de; ++l) gy = cadd(gy, cmul(Gs[(rr) * DS + l], Ys[(l) * DS + k]));
            abar = cscale(gy, wl[rr]);
          } else {
            abar = Y[m * D + k];
          }
          out = cadd(out, cscale(abar, wl[rr]));
          wsum += cmulc(abar, Gs[(rr) * DS + k]).x;
        }
        st.gbar[ro + (int64_t)k * S.sq] = out;
      }
    }
    wsum = group_sum_dpp(wsum, 4);
    if (kq == 0 && rr < rows) wb[rr] = wsum;
  }
  __syncthreads();
  // w-bar per row (w = l1[o1] l2[o2]) for k_adj_lbar, which folds it into the other legs' lambda-bar
  double* wrow = st.wbar + ((int64_t)slot * 4 + sp) * D * D;
  for (int idx = tid; idx < rows; idx += blockDim.x) wrow[row0 + idx] = wb[idx];
}

// lambda-bar of the other legs of one end (slot, side) from the per-row w-bar of both slices:
//   lambda-bar[f1][o1] += sum_p sum_o2 wbar[p][o1 d2 + o2] l2[o2],
//   lambda-bar[f2][o2] += sum_p sum_o1 wbar[p][o1 d2 + o2] l1[o1],
// summed in a fixed order.  An edge f gets such terms from the ends at its two vertices; pass 0
// adds the term of its lower vertex, pass 1 that of its higher one, so the additions into
// lambda-bar[f] happen in one order on every run.
__global__ __launch_bounds__(256) void k_adj_lbar(DevState st, const int32_t* __restrict__ items, int first,
                                                  int pass) {
  const int slot = blockIdx.x >> 1, side = blockIdx.x & 1;
  const int e = items[first + slot];
  const SideInfo& S = st.edges[e].side[side];
  const int D = st.D;
  const int d1 = S.oth[0] >= 0 ? st.chi[S.oth[0]] : 1;
  const int d2 = S.oth[1] >= 0 ? st.chi[S.oth[1]] : 1;
  const double* l1 = S.oth[0] >= 0 ? st.lam + (int64_t)S.oth[0] * D : nullptr;
  const double* l2 = S.oth[1] >= 0 ? st.lam + (int64_t)S.oth[1] * D : nullptr;
  const double* w0 = st.wbar + ((int64_t)slot * 4 + side * 2 + 0) * D * D;
  const double* w1 = st.wbar + ((int64_t)slot * 4 + side * 2 + 1) * D * D;
  const int tid = threadIdx.x;
  for (int leg = 0; leg < 2; ++leg) {
    const int f = S.oth[leg];
    if (f < 0) continue;
    const bool lower = st.edges[f].side[0].goff == S.goff;
    if (lower != (pass == 0)) continue;
    const int n = leg == 0 ? d1 : d2;
    for (int o = tid; o < n; o += blockDim.x) {
      double acc = 0.0;
      if (leg == 0) {
        for (int o2 = 0; o2 < d2; ++o2) {
          const int m = o * d2 + o2;
          acc += (w0[m] + w1[m]) * (l2 ? l2[o2] : 1.0);
        }
      } else {
        for (int o1 = 0; o1 < d1; ++o1) {
          const int m = o1 * d2 + o;
          acc += (w0[m] + w1[m]) * (l1 ? l1[o1] : 1.0);
        }
      }
      if (acc != 0.0) st.lbar[(int64_t)f * D + o] += acc;
    }
  }
}

// dL/dtheta of every instance from the per-edge (theta_J) and per-chunk (theta_h) accumulators,
// each summed in a fixed order (thread stride, then a fixed tree).
__global__ __launch_bounds__(256) void k_adj_theta(DevState st, int n_chunks) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  double tj = 0.0, th = 0.0;
  for (int e = threadIdx.x; e < st.NE; e += 256)
    if (st.edges[e].inst == k) tj += st.gpart[e];
  for (int c = threadIdx.x; c < n_chunks; c += 256)
    if (st.verts[(int)(st.chunks[c] >> 32)].inst == k) th += st.gpart[st.NE + c];
  const double sj = block_sum<256>(tj, red);
  const double sh = block_sum<256>(th, red);
  if (threadIdx.x == 0) {
    st.thbar[2 * k + 0] = sh;
    st.thbar[2 * k + 1] = sj;
  }
}

// ------------------------------------------------------------------ launchers

template <typename CT>
static hipError_t adj_launch(int which, const DevState& st, const int32_t* items, int first, int count,
                             int blocks_per_slice, const void* aux, hipStream_t stream) {
  switch (which) {
    case 1:
      if (count <= 0) return hipSuccess;
      hipLaunchKernelGGL(k_adj_tbar<CT>, dim3(count * 4), dim3(256), 0, stream, st, items, first);
      break;
    case 2:
      if (count <= 0) return hipSuccess;
      hipLaunchKernelGGL((k_adj_small<std::is_same<CT, float2>::value>), dim3(count), dim3(256), 0, stream, st,
                         items, first, (double2*)aux);
      break;
    case 3:
      if (count <= 0) return hipSuccess;
      {
        const size_t lds = (size_t)(2 * st.D + 2 * kRowBlock) * (st.D + 1) * sizeof(double2);
        if (lds > 65536) {  // above 64 KB of dynamic LDS the kernel's limit has to be raised
          const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adj_rows<CT>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
          if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_adj_rows<CT>, dim3(row_grid(st, count, blocks_per_slice)), dim3(256), lds, stream, st, items, first,
                           blocks_per_slice, (const double2*)aux);
      }
      break;
    case 6:  // lambda-bar of the other legs, both passes, over `count` items starting at `first`
      if (count <= 0) return hipSuccess;
      hipLaunchKernelGGL(k_adj_lbar, dim3(count * 2), dim3(256), 0, stream, st, items, first, 0);
      hipLaunchKernelGGL(k_adj_lbar, dim3(count * 2), dim3(256), 0, stream, st, items, first, 1);
      break;
    case 7:  // dL/dtheta per instance from the accumulators; count = number of RX chunks
      if (st.n_inst <= 0) return hipSuccess;
      hipLaunchKernelGGL(k_adj_theta, dim3(st.n_inst), dim3(256), 0, stream, st, count);
      break;
    case 4:  // readout seed over all vertices
      hipLaunchKernelGGL(k_adj_readout<CT>, dim3(st.NV), dim3(256), 0, stream, st);
      break;
    case 5:  // RX adjoint over `count` chunks starting at `first`; aux = pre-RX site tensors
      if (count <= 0) return hipSuccess;
      hipLaunchKernelGGL(k_adj_rx<CT>, dim3(count), dim3(256), 0, stream, st, aux, first);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(int which, bool c128, const DevState& st, const int32_t* items, int first, int count,
                          int blocks_per_slice, const void* aux, hipStream_t stream) {
  return c128 ? adj_launch<double2>(which, st, items, first, count, blocks_per_slice, aux, stream)
              : adj_launch<float2>(which, st, items, first, count, blocks_per_slice, aux, stream);
}

hipError_t launch_checkpoint(const DevState& st, const void* src, void* dst, int64_t bytes, int64_t slot_bytes,
                             hipStream_t stream) {
  const int64_t n32 = bytes / 4;
  const int64_t blocks64 = (n32 + 255) / 256;
  const int blocks = (int)(blocks64 < 4096 ? (blocks64 > 0 ? blocks64 : 1) : 4096);
  hipLaunchKernelGGL(k_checkpoint, dim3(blocks), dim3(256), 0, stream, (const uint32_t*)src, (uint32_t*)dst, n32,
                     slot_bytes / 4, st.step_ctr, st.max_steps);
  return hipGetLastError();
}

hipError_t launch_mean_z(const DevState& st, int row, hipStream_t stream) {
  if (st.n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mean_z, dim3(st.n_inst), dim3(256), 0, stream, st, row);
  return hipGetLastError();
}

hipError_t launch_seed_mean(const DevState& st, hipStream_t stream) {
  if (st.NV <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_seed_mean, dim3((st.NV + 255) / 256), dim3(256), 0, stream, st);
  return hipGetLastError();
}

hipError_t launch_fill_d(double* p, int64_t n, hipStream_t stream) {
  const int64_t blocks64 = (n + 255) / 256;
  const int blocks = (int)(blocks64 < 4096 ? (blocks64 > 0 ? blocks64 : 1) : 4096);
  hipLaunchKernelGGL(k_fill_d, dim3(blocks), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

}  // namespace gpeps
