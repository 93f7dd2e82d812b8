// HIP kernels of the graph-PEPS simple update for gfx950 (CDNA4).
//
// One two-qubit gate on edge e = (i, j) is three launches over every
// (instance, edge) work item of a colour class (Method section: simple
// update with the lambda weights as environment, bond dimension chi = D):
//
//   k_absorb_qr   per (item, end, physical slice p): absorb the lambda
//                 weights of the other legs into Gamma^(p) and QR-reduce the
//                 resulting [M x D_e] matrix in float64 (Householder, rows
//                 streamed in chunks, R only);
//   k_theta_svd   per item: Theta' = R_i diag(lambda_e) R_j^T times the
//                 diagonal RZZ phase, one-sided Jacobi SVD in float64 held in
//                 LDS, truncation to <= D values with lambda_e <- s/||s||, and
//                 the small re-absorb matrices T (below);
//   k_reabsorb    per (item, end, slice, 64-row block): Gamma'^(p) = Gamma^(p) T^(p).
//
// Why per-slice QR and T.  RZZ is diagonal in (s, t), so the physical index of
// each end passes through the gate unchanged.  Reducing each physical slice
// A^(p) = Q^(p) R^(p) separately gives block-diagonal isometries, so the
// singular values and vectors of the two-site tensor equal those of the
// smaller Theta'[(a,s),(t,b)] = g(s,t) sum_k R_i^(s)[a,k] lambda_k R_j^(t)[b,k].
// The new tensor of end i, Q_i U with the environment divided out again,
// equals Gamma_i^(s) T_i^(s) with
//   T_i^(s)[k,k'] = lambda_k / sigma_k' * sum_{t,b} g(s,t) R_j^(t)[b,k] V[(t,b),k']
// (and T_j^(t) likewise from conj(U) and R_i), because Q^H A = R.  Q is never
// formed and no division by a neighbouring lambda is needed: the weights
// absorbed into A cancel exactly against the ones the simple update divides out.
//
// Remaining kernels: RX layer (Eq. 2), mean-field <Z> readout (lambda^2 on
// every leg), product-state reset (Eq. 3) and the history step counter.

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

__device__ __forceinline__ int64_t rbuf_off(const DevState& st, int slot, int side, int p) {
  return (((int64_t)slot * 2 + side) * 2 + p) * st.D * st.D;
}

// ------------------------------------------------------------------ K1: absorb + QR

// Workgroup of 256 threads: thread (c = tid / 8, g = tid % 8) owns column c
// of the current row chunk, rows g, g + 8, ... .  The chunk is stacked under
// the running upper-triangular R (kept in LDS) and reduced column by column
// with complex Householder reflectors P = I - tau v v^H, v = x - beta e_0,
// beta = -phase(x_0) ||x||.  A column whose chunk part is exactly zero is
// skipped, so exact zeros stay exact.
template <typename CT>
__global__ __launch_bounds__(256) void k_absorb_qr(DevState st, const int32_t* __restrict__ items, int first) {
  const int task = blockIdx.x;
  const int slot = task >> 2;
  const int side = (task >> 1) & 1;
  const int p = task & 1;
  const int e = items[first + slot];
  const EdgeInfo& E = st.edges[e];
  const SideGeom G = side_geom(st, E.side[side]);
  const int n = st.chi[e];
  const int M = G.d1 * G.d2;
  const CT* gam = reinterpret_cast<const CT*>(st.gamma);
  double2* R = st.rbuf + rbuf_off(st, slot, side, p);
  const int D = st.D;
  const int tid = threadIdx.x;

  if (M <= n) {  // no reduction: R = A (M x n)
    for (int idx = tid; idx < M * n; idx += blockDim.x) {
      const int m = idx / n, k = idx - (idx / n) * n;
      R[m * D + k] = cscale(to_d2(gam[G.addr(p, m, k)]), G.env(m));
    }
    return;
  }

  constexpr int RPT = kQrChunk / 8;  // rows per thread per chunk
  __shared__ double2 Rm[kMaxD][kMaxD + 1];
  __shared__ double2 vb[kQrChunk];
  __shared__ double2 sh_v0;
  __shared__ double sh_tau;
  __shared__ int sh_skip;

  const int c = tid >> 3;
  const int g = tid & 7;
  for (int idx = tid; idx < kMaxD * (kMaxD + 1); idx += blockDim.x) (&Rm[0][0])[idx] = make_double2(0.0, 0.0);
  __syncthreads();

  double2 x[RPT];
  for (int r0 = 0; r0 < M; r0 += kQrChunk) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int m = r0 + g + 8 * i;
      x[i] = (c < n && m < M) ? cscale(to_d2(gam[G.addr(p, m, c)]), G.env(m)) : make_double2(0.0, 0.0);
    }
    for (int j = 0; j < n; ++j) {
      if (c == j) {
        double s2 = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          s2 += cabs2(x[i]);
          vb[g + 8 * i] = x[i];
        }
        s2 = group_sum(s2, 8);
        if (g == 0) {
          if (s2 == 0.0) {
            sh_skip = 1;
          } else {
            const double2 alpha = Rm[j][j];
            const double aa = sqrt(cabs2(alpha));
            const double nu = sqrt(aa * aa + s2);
            const double2 ph = aa > 0.0 ? cscale(alpha, 1.0 / aa) : make_double2(1.0, 0.0);
            const double2 beta = cscale(ph, -nu);
            const double2 v0 = csub(alpha, beta);
            sh_v0 = v0;
            sh_tau = 2.0 / (cabs2(v0) + s2);
            sh_skip = 0;
            Rm[j][j] = beta;
          }
        }
      }
      __syncthreads();
      if (!sh_skip) {
        if (c > j && c < n) {
          const double2 v0 = sh_v0;
          double2 w = make_double2(0.0, 0.0);
#pragma unroll
          for (int i = 0; i < RPT; ++i) w = cadd(w, cmulc(vb[g + 8 * i], x[i]));
          if (g == 0) w = cadd(w, cmulc(v0, Rm[j][c]));
          w.x = group_sum(w.x, 8);
          w.y = group_sum(w.y, 8);
          const double2 f = cscale(w, sh_tau);
#pragma unroll
          for (int i = 0; i < RPT; ++i) x[i] = csub(x[i], cmul(vb[g + 8 * i], f));
          if (g == 0) Rm[j][c] = csub(Rm[j][c], cmul(v0, f));
        } else if (c == j) {
#pragma unroll
          for (int i = 0; i < RPT; ++i) x[i] = make_double2(0.0, 0.0);
        }
      }
      __syncthreads();
    }
  }
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int a = idx / n, k = idx - (idx / n) * n;
    R[a * D + k] = (k >= a) ? Rm[a][k] : make_double2(0.0, 0.0);
  }
}

// ------------------------------------------------------------------ K2: Theta + Jacobi SVD + truncation

__device__ __forceinline__ void tournament_pair(int np, int round, int k, int& p, int& q) {
  // circle method: player 0 fixed, players 1..np-1 rotate
  auto pos = [&](int i) { return i == 0 ? 0 : 1 + ((i - 1 + round) % (np - 1)); };
  p = pos(k);
  q = pos(np - 1 - k);
  if (p > q) { const int t = p; p = q; q = t; }
}

template <typename CT>
__global__ __launch_bounds__(256) void k_theta_svd(DevState st, const int32_t* __restrict__ items, int first) {
  constexpr int NMAX = 2 * kMaxD;  // 64
  __shared__ double2 B[NMAX][NMAX + 1];  // column-major: B[col][row]
  __shared__ double2 W[NMAX][NMAX + 1];  // accumulated rotations, column-major
  __shared__ double lam_old[kMaxD];
  __shared__ double sig[NMAX];
  __shared__ int perm[NMAX];
  __shared__ int sh_rot;
  __shared__ int sh_chi;
  __shared__ double sh_norm;

  const int slot = blockIdx.x;
  const int e = items[first + slot];
  const EdgeInfo& E = st.edges[e];
  const InstParam ip = st.inst[E.inst];
  const int D = st.D;
  const int tid = threadIdx.x;
  const int de = st.chi[e];
  double* lam_e = st.lam + (int64_t)e * D;

  int r[2];
  for (int sd = 0; sd < 2; ++sd) {
    const SideInfo& S = E.side[sd];
    const int d1 = S.oth[0] >= 0 ? st.chi[S.oth[0]] : 1;
    const int d2 = S.oth[1] >= 0 ? st.chi[S.oth[1]] : 1;
    r[sd] = min(d1 * d2, de);
  }
  const int ri = r[0], rj = r[1];
  const int m0 = 2 * ri, n0 = 2 * rj;
  const bool trans = n0 > m0;  // orthogonalise the shorter side
  const int mB = trans ? n0 : m0;
  const int nB = trans ? m0 : n0;
  const double2* Ri0 = st.rbuf + rbuf_off(st, slot, 0, 0);
  const double2* Ri1 = st.rbuf + rbuf_off(st, slot, 0, 1);
  const double2* Rj0 = st.rbuf + rbuf_off(st, slot, 1, 0);
  const double2* Rj1 = st.rbuf + rbuf_off(st, slot, 1, 1);

  if (tid < kMaxD) lam_old[tid] = tid < de ? lam_e[tid] : 0.0;
  __syncthreads();

  // Theta'[(s,a)][(t,b)] = g(s,t) sum_k R_i^(s)[a,k] lambda_k R_j^(t)[b,k]
  for (int idx = tid; idx < m0 * n0; idx += blockDim.x) {
    const int rho = idx / n0, kap = idx - (idx / n0) * n0;
    const int s = rho / ri, a = rho - s * ri;
    const int t = kap / rj, b = kap - t * rj;
    const double2* Ra = (s ? Ri1 : Ri0) + a * D;
    const double2* Rb = (t ? Rj1 : Rj0) + b * D;
    double2 acc = make_double2(0.0, 0.0);
    for (int k = 0; k < de; ++k) acc = cadd(acc, cscale(cmul(Ra[k], Rb[k]), lam_old[k]));
    acc = cmul(acc, gate_phase(ip, s, t));
    if (!trans) B[kap][rho] = acc;
    else B[rho][kap] = cconj(acc);
  }
  for (int idx = tid; idx < nB * nB; idx += blockDim.x) {
    const int cc = idx / nB, rr = idx - (idx / nB) * nB;
    W[cc][rr] = make_double2(cc == rr ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();

  // one-sided (Hestenes) Jacobi on the nB columns of B, parallel tournament order
  const int np = nB + (nB & 1);
  const int npairs = np / 2;
  int L = 64;
  while (L > 1 && L * npairs > (int)blockDim.x) L >>= 1;
  const int pair_id = tid / L;
  const int lane = tid - pair_id * L;
  const bool active = pair_id < npairs;
  const double tol = 2.220446049250313e-16 * (double)mB;
  int sweep = 0;
  bool converged = (nB < 2);
  for (; sweep < st.max_sweeps && !converged; ++sweep) {
    if (tid == 0) sh_rot = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      int p = 0, q = 0;
      if (active) tournament_pair(np, round, pair_id, p, q);
      const bool work = active && q < nB;
      double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
      if (work) {
        for (int rr = lane; rr < mB; rr += L) {
          const double2 bp = B[p][rr], bq = B[q][rr];
          al += cabs2(bp);
          be += cabs2(bq);
          const double2 gg = cmulc(bp, bq);
          gr += gg.x;
          gi += gg.y;
        }
      }
      // every lane of a pair group takes part in the reductions
      al = group_sum(al, L);
      be = group_sum(be, L);
      gr = group_sum(gr, L);
      gi = group_sum(gi, L);
      const double gabs = sqrt(gr * gr + gi * gi);
      if (work && gabs > tol * sqrt(al * be) && gabs > 0.0) {
        const double zeta = (be - al) / (2.0 * gabs);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t);
        const double sn = cs * t;
        const double2 ph = make_double2(gr / gabs, gi / gabs);  // e^{i phi}
        // b_p' = c b_p - s e^{-i phi} b_q ;  b_q' = s e^{i phi} b_p + c b_q
        const double2 sph = cscale(ph, sn);
        for (int rr = lane; rr < mB; rr += L) {
          const double2 bp = B[p][rr], bq = B[q][rr];
          B[p][rr] = csub(cscale(bp, cs), cmulc(sph, bq));
          B[q][rr] = cadd(cmul(sph, bp), cscale(bq, cs));
        }
        for (int rr = lane; rr < nB; rr += L) {
          const double2 wp = W[p][rr], wq = W[q][rr];
          W[p][rr] = csub(cscale(wp, cs), cmulc(sph, wq));
          W[q][rr] = cadd(cmul(sph, wp), cscale(wq, cs));
        }
        if (lane == 0) sh_rot = 1;
      }
      __syncthreads();
    }
    converged = (sh_rot == 0);
    __syncthreads();
  }
  if (!converged && tid == 0) flag_status(st.status, kStatusNoConverge);

  // singular values, stable descending order
  if (tid < nB) {
    double s2 = 0.0;
    for (int rr = 0; rr < mB; ++rr) s2 += cabs2(B[tid][rr]);
    sig[tid] = sqrt(s2);
  }
  __syncthreads();
  if (tid < nB) {
    const double sv = sig[tid];
    int rank = 0;
    for (int d = 0; d < nB; ++d) {
      const double sd = sig[d];
      rank += (sd > sv) || (sd == sv && d < tid);
    }
    perm[rank] = tid;
  }
  __syncthreads();
  if (tid == 0) {
    const double smax = sig[perm[0]];
    int keep = 0;
    for (int d = 0; d < nB; ++d) keep += sig[d] > st.trunc_rel * smax;
    int chi = keep < D ? keep : D;
    if (chi < 1) chi = 1;
    double nrm = 0.0;
    for (int k = 0; k < chi; ++k) nrm += sig[perm[k]] * sig[perm[k]];
    nrm = sqrt(nrm);
    if (!(smax > 0.0)) flag_status(st.status, kStatusZeroTheta);
    if (!isfinite(nrm)) flag_status(st.status, kStatusNonFinite);
    sh_chi = chi;
    sh_norm = nrm;
    st.meta[slot].de_old = de;
    st.meta[slot].chi_new = chi;
    st.chi[e] = chi;
  }
  __syncthreads();
  const int chi = sh_chi;
  if (tid < D) lam_e[tid] = tid < chi ? sig[perm[tid]] / sh_norm : 0.0;

  // re-absorb matrices T (see the header comment), stored [D][D] row k, column k'
  CT* T = reinterpret_cast<CT*>(st.tbuf);
  for (int idx = tid; idx < 4 * de * D; idx += blockDim.x) {
    const int which = idx / (de * D);  // 0,1: end i slices s; 2,3: end j slices t
    const int rem = idx - which * de * D;
    const int k = rem / D, kp = rem - (rem / D) * D;
    double2 acc = make_double2(0.0, 0.0);
    if (kp < chi) {
      const int col = perm[kp];
      const double inv = lam_old[k] / sig[col];
      if (which < 2) {
        const int s = which;
        for (int t = 0; t < 2; ++t) {
          const double2* Rb = t ? Rj1 : Rj0;
          const double2 gph = gate_phase(ip, s, t);
          double2 part = make_double2(0.0, 0.0);
          for (int b = 0; b < rj; ++b) {
            const int kap = t * rj + b;
            const double2 v = trans ? cscale(B[col][kap], 1.0 / sig[col]) : W[col][kap];
            part = cadd(part, cmul(Rb[b * D + k], v));
          }
          acc = cadd(acc, cmul(gph, part));
        }
      } else {
        const int t = which - 2;
        for (int s = 0; s < 2; ++s) {
          const double2* Ra = s ? Ri1 : Ri0;
          const double2 gph = gate_phase(ip, s, t);
          double2 part = make_double2(0.0, 0.0);
          for (int a = 0; a < ri; ++a) {
            const int rho = s * ri + a;
            const double2 u = trans ? W[col][rho] : cscale(B[col][rho], 1.0 / sig[col]);
            part = cadd(part, cmulc(u, Ra[a * D + k]));
          }
          acc = cadd(acc, cmul(gph, part));
        }
      }
      acc = cscale(acc, inv);
    }
    const int sd = which >> 1, pp = which & 1;
    T[rbuf_off(st, slot, sd, pp) + k * D + kp] = from_d2<CT>(acc);
  }
}

// ------------------------------------------------------------------ K3: re-absorb

template <typename CT>
__global__ __launch_bounds__(256) void k_reabsorb(DevState st, const int32_t* __restrict__ items, int first,
                                                  int blocks_per_slice) {
  const int task = blockIdx.x;
  const int slot = task / (4 * blocks_per_slice);
  const int rem = task - slot * 4 * blocks_per_slice;
  const int sp = rem / blocks_per_slice;  // side * 2 + slice
  const int rb = rem - sp * blocks_per_slice;
  const int side = sp >> 1, p = sp & 1;
  const int e = items[first + slot];
  const EdgeInfo& E = st.edges[e];
  const SideInfo& S = E.side[side];
  const int D = st.D;
  const int d1 = S.oth[0] >= 0 ? st.chi[S.oth[0]] : 1;
  const int d2 = S.oth[1] >= 0 ? st.chi[S.oth[1]] : 1;
  const int M = d1 * d2;
  const int row0 = rb * kRowBlock;
  if (row0 >= M) return;
  const int rows = min(kRowBlock, M - row0);
  const SlotMeta meta = st.meta[slot];
  const int de = meta.de_old;
  const int ncol = max(de, meta.chi_new);  // columns that may be non-zero before or after

  __shared__ CT Ts[kMaxD][kMaxD + 1];
  __shared__ CT Gs[kRowBlock][kMaxD + 1];
  CT* gam = reinterpret_cast<CT*>(st.gamma);
  const CT* T = reinterpret_cast<const CT*>(st.tbuf) + rbuf_off(st, slot, side, p);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < de * D; idx += blockDim.x) {
    const int k = idx / D, kp = idx - (idx / D) * D;
    Ts[k][kp] = T[k * D + kp];
  }
  const int64_t base = S.goff + p * S.pstride;
  for (int idx = tid; idx < rows * de; idx += blockDim.x) {
    const int rr = idx / de, k = idx - (idx / de) * de;
    const int m = row0 + rr;
    const int o1 = m / d2, o2 = m - (m / d2) * d2;
    Gs[rr][k] = gam[base + (int64_t)o1 * S.so[0] + (int64_t)o2 * S.so[1] + (int64_t)k * S.sq];
  }
  __syncthreads();
  for (int idx = tid; idx < rows * ncol; idx += blockDim.x) {
    const int rr = idx / ncol, kp = idx - (idx / ncol) * ncol;
    const int m = row0 + rr;
    const int o1 = m / d2, o2 = m - (m / d2) * d2;
    CT out;
    if constexpr (sizeof(CT) == sizeof(float2)) {
      float ax = 0.f, ay = 0.f;
      for (int k = 0; k < de; ++k) {
        const CT gv = Gs[rr][k], tv = Ts[k][kp];
        ax += (float)gv.x * (float)tv.x - (float)gv.y * (float)tv.y;
        ay += (float)gv.x * (float)tv.y + (float)gv.y * (float)tv.x;
      }
      out.x = ax;
      out.y = ay;
    } else {
      double ax = 0.0, ay = 0.0;
      for (int k = 0; k < de; ++k) {
        const CT gv = Gs[rr][k], tv = Ts[k][kp];
        ax += gv.x * tv.x - gv.y * tv.y;
        ay += gv.x * tv.y + gv.y * tv.x;
      }
      out.x = ax;
      out.y = ay;
    }
    gam[base + (int64_t)o1 * S.so[0] + (int64_t)o2 * S.so[1] + (int64_t)kp * S.sq] = out;
  }
}

// ------------------------------------------------------------------ RX layer

// Gamma_v[0] <- c Gamma_v[0] - i s Gamma_v[1];  Gamma_v[1] <- -i s Gamma_v[0] + c Gamma_v[1]
template <typename CT>
__global__ __launch_bounds__(256) void k_rx(DevState st, int chunk_first) {
  const int64_t ch = st.chunks[chunk_first + blockIdx.x];
  const int v = (int)(ch >> 32);
  const int cidx = (int)(ch & 0xffffffff);
  const VertexInfo& V = st.verts[v];
  const InstParam ip = st.inst[V.inst];
  int64_t ps = 1;
  for (int l = 0; l < V.deg; ++l) ps *= st.D;
  CT* gam = reinterpret_cast<CT*>(st.gamma) + V.goff;
  const int64_t i0 = (int64_t)cidx * 1024;
  const double c = ip.rx_c, s = ip.rx_s;
  for (int64_t i = i0 + threadIdx.x; i < i0 + 1024 && i < ps; i += blockDim.x) {
    const double2 a = to_d2(gam[i]);
    const double2 b = to_d2(gam[i + ps]);
    // -i s b = (s b.y, -s b.x)
    const double2 na = make_double2(c * a.x + s * b.y, c * a.y - s * b.x);
    const double2 nb = make_double2(s * a.y + c * b.x, -s * a.x + c * b.y);
    gam[i] = from_d2<CT>(na);
    gam[i + ps] = from_d2<CT>(nb);
  }
}

// ------------------------------------------------------------------ <Z> readout

template <typename CT>
__global__ __launch_bounds__(256) void k_expect_z(DevState st, int v_first, int record) {
  const int v = v_first + blockIdx.x;
  const VertexInfo& V = st.verts[v];
  const int D = st.D;
  __shared__ double lw[kMaxDeg][kMaxD];
  __shared__ double red0[256], red1[256];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kMaxDeg * D; idx += blockDim.x) {
    const int l = idx / D, k = idx - (idx / D) * D;
    double w = 1.0;
    if (l < V.deg) {
      const double x = st.lam[(int64_t)V.leg[l] * D + k];
      w = x * x;
    }
    lw[l][k] = w;
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
      const int k = (int)(rest % D);
      rest /= D;
      w *= lw[l][k];
    }
    r0 += cabs2(to_d2(gam[i])) * w;
    r1 += cabs2(to_d2(gam[i + ps])) * w;
  }
  red0[tid] = r0;
  red1[tid] = r1;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      red0[tid] += red0[tid + off];
      red1[tid] += red1[tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double a = red0[0], b = red1[0];
    const double zv = (a - b) / (a + b);
    if (!isfinite(zv)) flag_status(st.status, kStatusNonFinite);
    st.z[v] = zv;
    if (record) {
      const int row = *st.step_ctr;
      if (row < st.max_steps) st.hist[(int64_t)row * st.NV + v] = zv;
    }
  }
}

__global__ void k_step_done(DevState st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *st.step_ctr += 1;
}

// ------------------------------------------------------------------ product state |0...0>

template <typename CT>
__global__ __launch_bounds__(256) void k_fill_zero(void* p, int64_t n) {
  CT* a = reinterpret_cast<CT*>(p);
  const CT zero = from_d2<CT>(make_double2(0.0, 0.0));
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = zero;
}

template <typename CT>
__global__ __launch_bounds__(256) void k_reset(DevState st) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  CT* gam = reinterpret_cast<CT*>(st.gamma);
  for (int64_t v = gid; v < st.NV; v += stride) {
    gam[st.verts[v].goff] = from_d2<CT>(make_double2(1.0, 0.0));
    st.z[v] = 1.0;
  }
  for (int64_t i = gid; i < (int64_t)st.NE * st.D; i += stride) st.lam[i] = (i % st.D) == 0 ? 1.0 : 0.0;
  for (int64_t e = gid; e < st.NE; e += stride) st.chi[e] = 1;
  if (gid == 0) {
    *st.step_ctr = 0;
    *st.status = 0;
  }
}

// ------------------------------------------------------------------ host-side launchers

template <typename CT>
static hipError_t launch_set(int which, const DevState& st, const int32_t* items, int first, int count,
                             int blocks_per_slice, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  switch (which) {
    case 1:
      hipLaunchKernelGGL(k_absorb_qr<CT>, dim3(count * 4), dim3(256), 0, stream, st, items, first);
      break;
    case 2:
      hipLaunchKernelGGL(k_theta_svd<CT>, dim3(count), dim3(256), 0, stream, st, items, first);
      break;
    case 3:
      hipLaunchKernelGGL(k_reabsorb<CT>, dim3(count * 4 * blocks_per_slice), dim3(256), 0, stream, st, items,
                         first, blocks_per_slice);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gpeps

// C++ entry points used by the host driver (gpeps_host.cpp).
namespace gpeps {

hipError_t launch_edge_kernel(int which, bool c128, const DevState& st, const int32_t* items, int first, int count,
                              int blocks_per_slice, hipStream_t stream) {
  return c128 ? launch_set<double2>(which, st, items, first, count, blocks_per_slice, stream)
              : launch_set<float2>(which, st, items, first, count, blocks_per_slice, stream);
}

hipError_t launch_rx(bool c128, const DevState& st, int chunk_first, int n_chunks, hipStream_t stream) {
  if (n_chunks <= 0) return hipSuccess;
  if (c128) hipLaunchKernelGGL(k_rx<double2>, dim3(n_chunks), dim3(256), 0, stream, st, chunk_first);
  else hipLaunchKernelGGL(k_rx<float2>, dim3(n_chunks), dim3(256), 0, stream, st, chunk_first);
  return hipGetLastError();
}

hipError_t launch_expect_z(bool c128, const DevState& st, int v_first, int n_verts, int record, hipStream_t stream) {
  if (n_verts <= 0) return hipSuccess;
  if (c128) hipLaunchKernelGGL(k_expect_z<double2>, dim3(n_verts), dim3(256), 0, stream, st, v_first, record);
  else hipLaunchKernelGGL(k_expect_z<float2>, dim3(n_verts), dim3(256), 0, stream, st, v_first, record);
  return hipGetLastError();
}

hipError_t launch_step_done(const DevState& st, hipStream_t stream) {
  hipLaunchKernelGGL(k_step_done, dim3(1), dim3(64), 0, stream, st);
  return hipGetLastError();
}

hipError_t launch_reset(bool c128, const DevState& st, int64_t n_gamma, hipStream_t stream) {
  const int64_t blocks64 = (n_gamma + 255) / 256;
  const int blocks = (int)(blocks64 < 65536 ? (blocks64 > 0 ? blocks64 : 1) : 65536);
  if (c128) {
    hipLaunchKernelGGL(k_fill_zero<double2>, dim3(blocks), dim3(256), 0, stream, st.gamma, n_gamma);
    hipLaunchKernelGGL(k_reset<double2>, dim3(256), dim3(256), 0, stream, st);
  } else {
    hipLaunchKernelGGL(k_fill_zero<float2>, dim3(blocks), dim3(256), 0, stream, st.gamma, n_gamma);
    hipLaunchKernelGGL(k_reset<float2>, dim3(256), dim3(256), 0, stream, st);
  }
  return hipGetLastError();
}

}  // namespace gpeps
