// HIP kernels of the graph-PEPS simple update for gfx950 (CDNA4).
//
// One two-qubit gate on edge e = (i, j) is three launches over every
// (instance, edge) work item of a colour class (Method section: simple
// update with the lambda weights as environment, bond dimension chi = D):
//
//   k_absorb_gram per (item, end, physical slice p): absorb the lambda weights
//   / k_absorb_qr of the other legs into Gamma^(p) and reduce the resulting
//                 [M x D_e] matrix A to an R factor with R^H R = A^H A in
//                 float64: Gram matrix on the matrix cores + Cholesky for
//                 complex64 storage, Householder (rows streamed in chunks, R
//                 only) for complex128;
//   k_theta_svd   per item: Theta' = R_i diag(lambda_e) R_j^T times the
//                 diagonal RZZ phase, one-sided Jacobi SVD in float64 held in
//                 LDS, truncation to <= D values with lambda_e <- s/||s||, and
//                 the small re-absorb matrices T (below);
//   k_reabsorb_mfma / k_reabsorb  per (item, end, slice, row block):
//                 Gamma'^(p) = Gamma^(p) T^(p).
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

#include "gpeps_device.h"
#include "gpeps_internal.h"

namespace gpeps {

hipError_t launch_svd_big(bool c128, const DevState& st, const int32_t* items, int first, int count,
                          hipStream_t stream);

// ------------------------------------------------------------------ K1: absorb + QR

// Workgroup of 256 threads for at most NC columns: lane group c = tid / (256 / NC) owns
// column c of the current row chunk, lane g of the group rows g, g + 256 / NC, ... .  The
// chunk is stacked under the running upper-triangular R (kept in LDS) and reduced column by
// column with complex Householder reflectors P = I - tau v v^H, v = x - beta e_0,
// beta = -phase(x_0) ||x||.  One barrier per column: the group of column j + 1 publishes its
// chunk rows (already updated by reflector j) and their squared norm while the others apply
// reflector j, and every group rebuilds reflector j + 1 from that copy (bit-identical in all
// groups).  A column whose chunk part is exactly zero is skipped, so exact zeros stay exact.
template <typename CT, int NC, int RPT>
__global__ __launch_bounds__(256) void k_absorb_qr(DevState st, const int32_t* __restrict__ items, int first) {
  constexpr int LPC = 256 / NC;  // lanes per column (RPT: rows per lane per chunk)
  constexpr int CH = LPC * RPT;  // rows per chunk
  int slot, side, p;
  end_task(st, blockIdx.x, slot, side, p);
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

  __shared__ double2 Rm[NC][NC + 1];
  __shared__ double2 vb[2][CH];  // chunk rows of the next pivot column, by step parity
  __shared__ double vn[2];        // and their squared norm

  const int c = tid / LPC;
  const int g = tid - (tid / LPC) * LPC;
  for (int idx = tid; idx < NC * (NC + 1); idx += blockDim.x) (&Rm[0][0])[idx] = make_double2(0.0, 0.0);

  double2 x[RPT];
  for (int r0 = 0; r0 < M; r0 += CH) {
    // every load of the chunk is issued before the first use: addresses are clamped into the
    // matrix and rows or columns outside it are zeroed afterwards
    const int cc = c < n ? c : n - 1;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int m = r0 + g + LPC * i;
      const int mc = m < M ? m : M - 1;
      const double2 a = cscale(to_d2(gam[G.addr(p, mc, cc)]), G.env(mc));
      x[i] = (c < n && m < M) ? a : make_double2(0.0, 0.0);
    }
    if (c == 0) {
      double sp = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        vb[0][g + LPC * i] = x[i];
        sp += cabs2(x[i]);
      }
      sp = group_sum_dpp(sp, LPC);
      if (g == 0) vn[0] = sp;
    }
    bool set_diag = false;  // this group's column got a new diagonal in this chunk
    double2 my_beta = make_double2(0.0, 0.0);
    __syncthreads();
    for (int j = 0; j < n; ++j) {
      const double2* vj = vb[j & 1];
      const double2 alpha = Rm[j][j];
      double2 v[RPT];
#pragma unroll
      for (int i = 0; i < RPT; ++i) v[i] = vj[g + LPC * i];
      const double s2 = vn[j & 1];  // squared norm of the pivot column's chunk part
      if (s2 > 0.0) {
        const double aa2 = cabs2(alpha);
        const double nu2 = aa2 + s2;
        const double nu = nu2 * rsq_nr(nu2);
        const double2 ph = aa2 > 0.0 ? cscale(alpha, rsq_nr(aa2)) : make_double2(1.0, 0.0);
        const double2 beta = cscale(ph, -nu);
        const double2 v0 = csub(alpha, beta);
        const double tau = 2.0 * rcp_nr(cabs2(v0) + s2);
        if (c == j) {
          set_diag = true;
          my_beta = beta;
        } else if (c > j && c < n) {
          double wr = 0.0, wi = 0.0;
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            const double2 t = cmulc(v[i], x[i]);
            wr += t.x;
            wi += t.y;
          }
          double2 rjc = make_double2(0.0, 0.0);
          if (g == 0) {
            rjc = Rm[j][c];
            const double2 t = cmulc(v0, rjc);
            wr += t.x;
            wi += t.y;
          }
          group_sum2_dpp(wr, wi, LPC);
          const double2 f = make_double2(wr * tau, wi * tau);
#pragma unroll
          for (int i = 0; i < RPT; ++i) x[i] = csub(x[i], cmul(v[i], f));
          if (g == 0) Rm[j][c] = csub(rjc, cmul(v0, f));
        }
      }
      if (c == j + 1) {
        double sp = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          vb[(j + 1) & 1][g + LPC * i] = x[i];
          sp += cabs2(x[i]);
        }
        sp = group_sum_dpp(sp, LPC);
        if (g == 0) vn[(j + 1) & 1] = sp;
      }
      __syncthreads();
    }
    if (set_diag && g == 0) Rm[c][c] = my_beta;
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int a = idx / n, k = idx - (idx / n) * n;
    R[a * D + k] = (k >= a) ? Rm[a][k] : make_double2(0.0, 0.0);
  }
}

// ------------------------------------------------------------------ K1 (complex64): absorb + Gram / Cholesky

// Complex64 storage takes R from the Gram matrix: G = A^H A (A = Gamma^(p) with the other legs'
// lambdas on its rows) on the FP64 matrix cores, then R^H R = G by Cholesky.  Only R^H R enters
// the update (the spectrum of Theta' and the new tensors are unchanged by R -> W R, W unitary),
// so this R serves as the Householder one does.  With v_mfma_f64_16x16x4f64 lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[l / 16 + 4 r][l % 16]; the reduction
// index (the row m of A) is l / 16, so a lane holds A[m][k] for one column k of each 16-column
// tile and the same registers serve both operands.  Each wave sums a quarter of the rows; the
// four partial Gram matrices are added in LDS in a fixed order.  G rounds at ~2^-53 ||A||^2:
// directions of A below ~1e-7 of its norm are not resolved, about the complex64 rounding of the
// stored tensors, and a Cholesky pivot below 1e-13 of its column's squared norm is taken as
// zero (that row of R is zero), which keeps exact zeros exact.
template <int NC>
__global__ __launch_bounds__(256, NC == 32 ? 4 : 1) void k_absorb_gram(DevState st, const int32_t* __restrict__ items, int first) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int NT16 = NC / 16;                 // column tiles of 16
  constexpr int NTILE = NT16 * (NT16 + 1) / 2;  // tiles on and above the diagonal
  constexpr int UNR = NT16 >= 4 ? 2 : 4 / NT16;  // row steps (of 4 rows) per load batch in flight
  int slot, side, p;
  end_task(st, blockIdx.x, slot, side, p);
  const int e = items[first + slot];
  const EdgeInfo& E = st.edges[e];
  const SideGeom G = side_geom(st, E.side[side]);
  const int n = st.chi[e];
  const int M = G.d1 * G.d2;
  const float2* gam = reinterpret_cast<const float2*>(st.gamma);
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

  // LDS: the partial tiles of waves 2 and 3 (part0 | part1), then the upper triangle of G,
  // which overlaps part1 only: part1 is dead once wave 1 has added it, and wave 0 reads part0
  // while it writes G.
  constexpr int PART = NTILE * 4 * 64;
  constexpr int GSZ = NC * (NC + 1);
  __shared__ double2 lds[PART + (GSZ > PART ? GSZ : PART)];
  __shared__ double dg[NC];           // squared column norms (diagonal of G)
  __shared__ double envs[2][NC];      // lambda weights of the other two legs (1 for a missing leg)
  double2* part0 = lds;
  double2* part1 = lds + PART;
  auto Gs = [&](int i, int j) -> double2& { return lds[PART + i * (NC + 1) + j]; };

  if (tid < NC) {
    envs[0][tid] = (G.l1 && tid < G.d1) ? G.l1[tid] : 1.0;
    envs[1][tid] = (G.l2 && tid < G.d2) ? G.l2[tid] : 1.0;
  }
  __syncthreads();

  const int l = tid & 63, wv = tid >> 6, li = l & 15, lk = l >> 4;
  d4 gr[NTILE], gi[NTILE];
#pragma unroll
  for (int t = 0; t < NTILE; ++t) {
    gr[t] = (d4){0.0, 0.0, 0.0, 0.0};
    gi[t] = (d4){0.0, 0.0, 0.0, 0.0};
  }
  // Software pipelined: the complex64 elements of the next batch of rows (4 ks + l / 16, columns
  // 16 t + l % 16) are in flight while the products of the current batch run.  A row past the
  // end gets weight 0 (its load is clamped to the last row).
  const int ksteps = (M + 3) >> 2;
  const int64_t pbase = G.base + p * G.pstride;
  float2 nx[UNR][NT16];
  double nw[UNR];
  auto fetch = [&](int ks0) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int m = 4 * (ks0 + 4 * u) + lk;
      const bool mv = m < M;
      const int mc = mv ? m : M - 1;
      const int o1 = mc / G.d2, o2 = mc - (mc / G.d2) * G.d2;
      nw[u] = mv ? envs[0][o1] * envs[1][o2] : 0.0;
      const int64_t ro = pbase + (int64_t)o1 * G.s1 + (int64_t)o2 * G.s2;
#pragma unroll
      for (int t = 0; t < NT16; ++t) {
        const int k = 16 * t + li;
        const int kc = k < n ? k : n - 1;
        nx[u][t] = gam[ro + (int64_t)kc * G.sq];
      }
    }
  };
  fetch(wv);
  for (int ks0 = wv; ks0 < ksteps; ks0 += 4 * UNR) {
    float2 x[UNR][NT16];
    double w[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      w[u] = nw[u];
#pragma unroll
      for (int t = 0; t < NT16; ++t) x[u][t] = nx[u][t];
    }
    if (ks0 + 4 * UNR < ksteps) fetch(ks0 + 4 * UNR);
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      double2 a[NT16];
#pragma unroll
      for (int t = 0; t < NT16; ++t) {
        const double wt = 16 * t + li < n ? w[u] : 0.0;
        a[t] = make_double2(wt * (double)x[u][t].x, wt * (double)x[u][t].y);
      }
      int tile = 0;
#pragma unroll
      for (int ta = 0; ta < NT16; ++ta)
#pragma unroll
        for (int tb = ta; tb < NT16; ++tb) {
          // G[k][k'] = sum_m conj(A[m][k]) A[m][k']: Re = Ar^T Ar + Ai^T Ai, Im = Ar^T Ai - Ai^T Ar.
          // On a diagonal tile the second term of Im is the transpose of the first, so only
          // X = Ar^T Ai is accumulated there and Im = X - X^T is formed once, after the sum.
          gr[tile] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].x, a[tb].x, gr[tile], 0, 0, 0);
          gr[tile] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].y, a[tb].y, gr[tile], 0, 0, 0);
          gi[tile] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta].x, a[tb].y, gi[tile], 0, 0, 0);
          if (ta != tb) gi[tile] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[ta].y, a[tb].x, gi[tile], 0, 0, 0);
          ++tile;
        }
    }
  }
  // partial sums of the four waves, added in a fixed order: (0 + 2) + (1 + 3)
  if (wv >= 2) {
    double2* part = wv == 2 ? part0 : part1;
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) part[(t * 4 + r) * 64 + l] = make_double2(gr[t][r], gi[t][r]);
  }
  __syncthreads();
  if (wv < 2) {
    const double2* part = wv == 0 ? part0 : part1;
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double2 q = part[(t * 4 + r) * 64 + l];
        gr[t][r] += q.x;
        gi[t][r] += q.y;
      }
  }
  __syncthreads();
  if (wv == 1) {
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) part0[(t * 4 + r) * 64 + l] = make_double2(gr[t][r], gi[t][r]);
  }
  __syncthreads();
  if (wv == 0) {
    int tile = 0;
#pragma unroll
    for (int ta = 0; ta < NT16; ++ta)
#pragma unroll
      for (int tb = ta; tb < NT16; ++tb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double2 q = part0[(tile * 4 + r) * 64 + l];
          const double2 v = make_double2(gr[tile][r] + q.x, gi[tile][r] + q.y);
          // off the diagonal tiles k < k' always; a diagonal tile is stored whole (its lower
          // half holds X[k'][k] for the antisymmetrisation below)
          Gs(16 * ta + lk + 4 * r, 16 * tb + li) = v;
        }
        ++tile;
      }
  }
  __syncthreads();
  // Im G on the diagonal tiles: X[k][k'] - X[k'][k] on the upper triangle (which is all the
  // factorisation reads), exactly 0 on the diagonal; only the upper entries are written
  for (int idx = tid; idx < NT16 * 256; idx += blockDim.x) {
    const int t16 = 16 * (idx >> 8), k = t16 + ((idx >> 4) & 15), kp = t16 + (idx & 15);
    if (k < kp) Gs(k, kp).y -= Gs(kp, k).y;
    else if (k == kp) Gs(k, k).y = 0.0;
  }
  if (tid < n) dg[tid] = Gs(tid, tid).x;
  __syncthreads();
  if constexpr (NC == 16) {
    // One wave, no barriers: lane l holds column j = l % 16 of the upper triangle, rows
    // i = l / 16 + 4 r (r = 0..3); the pivot comes by readlane and row k of R through LDS
    // (same wave, so the write precedes the reads).  The arithmetic is that of the loop below.
    __shared__ double2 rowk[2][16];
    if (wv != 0) return;
    const int j = l & 15, rq = l >> 4;
    double2 gq[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = rq + 4 * r;
      const double2 t = Gs(i, j);
      gq[r] = (i <= j && j < n) ? t : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if (k < n) {
        const double d = readlane_d(gq[k >> 2].x, k + 16 * (k & 3));  // G[k][k]
        const bool keep = d > 1e-13 * dg[k];
        const double rk = keep ? rsq_nr(d) : 0.0;  // 1 / R[k][k]
        if (rq == (k & 3) && j >= k) {
          const double2 v = j == k ? make_double2(keep ? d * rk : 0.0, 0.0) : cscale(gq[k >> 2], rk);
          gq[k >> 2] = v;
          rowk[k & 1][j] = v;
        }
        wave_lds_sync();  // other lanes read what these lanes wrote
        const double2 rkj = rowk[k & 1][j];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = rq + 4 * r;
          const double2 rki = rowk[k & 1][i];
          if (i > k && i <= j && j < n) gq[r] = csub(gq[r], cmulc(rki, rkj));
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = rq + 4 * r;
      if (i < n && j < n) R[i * D + j] = j >= i ? gq[r] : make_double2(0.0, 0.0);
    }
    return;
  }
  // right-looking Cholesky, R^H R = G, R upper triangular, in place in the upper triangle
  for (int k = 0; k < n; ++k) {
    const double d = Gs(k, k).x;
    const bool keep = d > 1e-13 * dg[k];
    const double rk = keep ? rsq_nr(d) : 0.0;  // 1 / R[k][k]
    __syncthreads();
    if (tid >= k && tid < n) Gs(k, tid) = tid == k ? make_double2(keep ? d * rk : 0.0, 0.0) : cscale(Gs(k, tid), rk);
    __syncthreads();
    const int w = n - k - 1;
    for (int idx = tid; idx < w * w; idx += blockDim.x) {
      const int i = k + 1 + idx / w, j = k + 1 + idx - (idx / w) * w;
      if (i <= j) Gs(i, j) = csub(Gs(i, j), cmulc(Gs(k, i), Gs(k, j)));
    }
    __syncthreads();
  }
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int a = idx / n, k = idx - (idx / n) * n;
    R[a * D + k] = (k >= a) ? Gs(a, k) : make_double2(0.0, 0.0);
  }
}

// ------------------------------------------------------------------ K2: Theta + Jacobi SVD + truncation

// One workgroup of NT = 256 threads per item; NMAX = 2 * largest D handled
// (32 for D <= 16, 64 for D <= 32).  Theta' lives in LDS as the matrix B whose
// columns are orthogonalised: B = Theta' when Theta' has no more columns than
// rows, else B = Theta'^H.  One-sided (Hestenes) Jacobi rotates column pairs
// in a parallel tournament order (complex64: columns held in registers, see the
// loop; complex128: circle method through LDS); squared column norms are tracked
// and recomputed at the start of every sweep, so each rotation needs a single
// reduction (the inner product).  A pair is rotated when its inner product
// exceeds 2^-52 * mB relative to the column norms and also exceeds
// 2^-52 * eps^2 * ||B||_F^2 (eps = truncation cutoff): pairs below that are
// made of columns far under the cutoff (rounding noise), whose rotation
// cannot move a kept singular vector.  The sweep loop ends when a sweep
// applies no rotation, or (complex64 path) when every rotation of the sweep
// had |g|^2 <= 1e-8 al be (angles below 1e-4): by the quadratic convergence of
// the sweeps the off-diagonal left is then O(1e-8) relative, under the 2^-24
// rounding of the complex64 tensors the update writes.  The complex64 path also takes one Newton step, not
// two, for the reciprocal square roots (unitarity to ~1e-13 per rotation), and runs the
// iteration on X = R^H, R from a column-pivoted Cholesky factorisation of B^H B (below), whose
// columns start nearly orthogonal and graded.
// ACC (complex128 path) also accumulates the rotations W, which give the
// other set of singular vectors directly; without it (complex64 path, cutoff
// ~1e-6) they are recovered from the original Theta' as U = Theta' V / sigma
// or V = Theta'^H U / sigma, accurate to ~2^-52 sigma_0 / sigma_k, well below
// the complex64 storage rounding for every kept value.
// BWD: the forward update (the same path and arithmetic, so the truncation rank and the
// gauge of the new tensors are the forward ones bit for bit) that also keeps what the
// reverse sweep needs: every singular triplet (bU, bV, bS) and float64 T matrices (t64).
constexpr double kJacobiQuiet = 1e-12;     // (1e-6)^2: relative size of a "small" rotation
constexpr double kJacobiQuietC64 = 1e-8;   // (1e-4)^2: the same for the complex64 path

template <typename CT, int NT, int NMAX, bool ACC_, bool BWD = false>
__global__ __launch_bounds__(NT, (NMAX == 64 && !ACC_) ? 2 : 1) void k_theta_svd(DevState st, const int32_t* __restrict__ items, int first) {
  constexpr bool ACC = ACC_;
  constexpr int DM = NMAX / 2;             // largest bond dimension handled
  constexpr int EPT = NMAX * NMAX / NT;    // Theta' entries per thread (16)
  constexpr int RPT = NMAX * DM / NT;      // singular-vector entries per thread (8)
  constexpr int KPT = (DM * DM + NT - 1) / NT;  // (k, k') pairs per thread (4)
  constexpr int RPL = NMAX * NMAX / (2 * NT);  // rows per lane of a Jacobi column pair (upper bound)
  static_assert(2 * NT / NMAX <= 64 && RPL * (2 * NT / NMAX) >= NMAX, "Jacobi rows must fit RPL per lane");
  constexpr bool PRE = !ACC;               // Cholesky preconditioning (complex64 path)
  constexpr int DS = DM + 1;               // padded row stride of the staging arena (no bank conflicts)
  // B: column-major B[col][row], column stride NMAX (a 16-lane group reading 16 consecutive rows
  // covers all 64 LDS banks once; lane groups that share an LDS cycle start on different row
  // blocks, below).  The same memory is the staging arena of 4 DM DS elements.
  constexpr int kBsz = NMAX * NMAX > 4 * DM * DS ? NMAX * NMAX : 4 * DM * DS;
  __shared__ double2 Bmem[kBsz];
  __shared__ double2 Wmem[ACC ? kBsz : 1];  // accumulated rotations W[col][row] (ACC only), also an arena
  double2 (*const B)[NMAX] = reinterpret_cast<double2 (*)[NMAX]>(Bmem);
  double2 (*const W)[NMAX] = reinterpret_cast<double2 (*)[NMAX]>(Wmem);
  __shared__ double nrm[NMAX];
  __shared__ double lam_old[kMaxD];
  __shared__ double sig[NMAX];
  __shared__ int perm[NMAX];
  __shared__ int sh_rot, sh_big;
  __shared__ int sh_chi;
  __shared__ double sh_norm;
  __shared__ double sh_floor;
  __shared__ int colid[NMAX];   // original column of each pivoted position
  __shared__ double red_w[NT / 64];      // per-wave partial sums
  double2* const arena = Bmem;
  double2* const A0 = arena;            // [2 DM DS]
  double2* const A1 = arena + 2 * DM * DS;  // [2 DM DS]

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
  const double2* Rg = st.rbuf + rbuf_off(st, slot, 0, 0);  // 4 consecutive [D][D] blocks: i0, i1, j0, j1

  // stage the R factors of one end ([2][r][de], row stride DS) into an LDS region
  auto stage_r = [&](double2* dst, int side, int rows) {
    for (int idx = tid; idx < 2 * rows * de; idx += NT) {
      const int sl = idx / (rows * de);
      const int rem = idx - sl * rows * de;
      const int rr = rem / de, k = rem - (rem / de) * de;
      dst[sl * DM * DS + rr * DS + k] = Rg[(int64_t)(side * 2 + sl) * D * D + rr * D + k];
    }
  };

  if (tid < kMaxD) lam_old[tid] = tid < de ? lam_e[tid] : 0.0;

  // Theta'[(s,a)][(t,b)] = g(s,t) sum_k R_i^(s)[a,k] lambda_k R_j^(t)[b,k]: the complex product
  // [2 r_i x D_e] [D_e x 2 r_j] on v_mfma_f64_16x16x4f64, four real products per complex one,
  // operands straight from the R factors in global memory.  With that instruction lane l holds
  // A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[l / 16 + 4 r][l % 16], r = 0..3.
  // Each wave takes 16 x 16 output tiles; ||Theta'||_F^2 is reduced on the way.
  {
    typedef double d4 __attribute__((ext_vector_type(4)));
    constexpr int KS = DM / 4;  // k steps of 4 at the largest bond
    const int l = tid & 63, wv = tid >> 6, li = l & 15, lk = l >> 4;
    const int tiles_c = (n0 + 15) >> 4;
    const int ntiles = ((m0 + 15) >> 4) * tiles_c;
    const int ksteps = (de + 3) >> 2;
    double fro = 0.0;
    for (int tile = wv; tile < ntiles; tile += NT / 64) {
      const int tr = tile / tiles_c, tc = tile - (tile / tiles_c) * tiles_c;
      const int rho = 16 * tr + li, kap = 16 * tc + li;
      const bool rv = rho < m0, cv = kap < n0;
      const int s = rv ? rho / ri : 0, a = rv ? rho - s * ri : 0;
      const int t = cv ? kap / rj : 0, b = cv ? kap - t * rj : 0;
      const double2* Ra = Rg + (int64_t)s * D * D + a * D;
      const double2* Rb = Rg + (int64_t)(2 + t) * D * D + b * D;
      double2 x[KS], y[KS];
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const int k = 4 * kk + lk;
        x[kk] = (rv && k < de) ? cscale(Ra[k], lam_e[k]) : make_double2(0.0, 0.0);
        y[kk] = (cv && k < de) ? Rb[k] : make_double2(0.0, 0.0);
      }
      // The registers x, y serve C = X Y (A = X, B = Y) and C^T = Y^T X^T (A = Y^T, B = X^T)
      // alike; the orientation is chosen so that the 16 lanes sharing an output register
      // store 16 consecutive rows of one column of B.
      d4 cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        if (kk < ksteps) {
          // trans: A = X, B = Y (lanes l % 16 <-> kap); else A = Y^T, B = X^T (lanes <-> rho)
          const double2 a = trans ? x[kk] : y[kk];
          const double2 b = trans ? y[kk] : x[kk];
          cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cr, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, ci, 0, 0, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ro = trans ? 16 * tr + lk + 4 * r : rho;  // row of Theta'
        const int co = trans ? kap : 16 * tc + lk + 4 * r;  // column of Theta'
        if (ro < m0 && co < n0) {
          const double2 v = cmul(make_double2(cr[r], ci[r]), gate_phase(ip, ro / ri, co / rj));
          fro += cabs2(v);
          if (!trans) B[co][ro] = v;
          else B[ro][co] = cconj(v);
          // the reverse sweep recovers the other vector set through Theta' (kept row-major)
          if (BWD && !ACC) st.wsb[(int64_t)slot * adj_scratch(D) + (int64_t)32 * D * D + ro * 2 * D + co] = v;
        }
      }
    }
    fro = group_sum_dpp(fro, 64);
    if (l == 0) red_w[wv] = fro;
  }
  if (ACC) {
    for (int idx = tid; idx < nB * nB; idx += NT) {
      const int cc = idx / nB, rr = idx - (idx / nB) * nB;
      W[cc][rr] = make_double2(cc == rr ? 1.0 : 0.0, 0.0);
    }
  }
  __syncthreads();
  if (tid == 0) {
    double f = 0.0;
    for (int w = 0; w < NT / 64; ++w) f += red_w[w];
    sh_floor = f * st.trunc_rel * st.trunc_rel * 2.220446049250313e-16;
  }

  // Preconditioning (complex64 path): R from a column-pivoted Cholesky factorisation of the
  // Gram matrix, P^T B^H B P = R^H R, then the Jacobi iteration runs on X = R^H (nB x nB).  With
  // Q = B P R^-1 (orthonormal columns), B P = Q R and X = U_X S W^H gives B = (Q W) S (P U_X)^H,
  // so the orthogonalised columns of X are B's right singular vectors (rows permuted by P) and
  // Q is never needed.  Only R^H R enters, as for the R factors of the absorb kernel: directions
  // of B below ~1e-8 of its norm are not resolved, two orders under the truncation cutoff and
  // about the complex64 rounding of the stored tensors; the factorisation stops at a pivot below
  // 64 eps of the first (the remaining rows of R are zero).
  int mJ = mB;
  if (PRE) {
    // G = B^H B on the FP64 matrix cores, 16 x 16 tiles over the waves (tile wv + q NW of the
    // tg x tg grid to wave wv; lane l holds rows i0 + l / 16 + 4 r, column j0 + l % 16 of each).
    constexpr int NW = NT / 64;
    constexpr int TPW = ((NMAX / 16) * (NMAX / 16) + NW - 1) / NW;  // tiles per wave (at most)
    const int wv = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int tg = (nB + 15) >> 4;
    cgemm_d4 sr[TPW], si[TPW];
    {
      auto fa = [&](int i, int k) -> double2 {
        return (i < nB && k < mB) ? cconj(B[i][k]) : make_double2(0.0, 0.0);
      };
      auto fb = [&](int k, int jj) -> double2 {
        return (k < mB && jj < nB) ? B[jj][k] : make_double2(0.0, 0.0);
      };
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        const int tile = wv + q * NW;
        if (tile < tg * tg) cgemm_tile(16 * (tile / tg), 16 * (tile - (tile / tg) * tg), mB, fa, fb, sr[q], si[q]);
      }
    }
    auto tile_ij = [&](int q, int& ti, int& tj) {
      const int tile = wv + q * NW;
      ti = tile / tg;
      tj = tile - ti * tg;
      return tile < tg * tg;
    };
    __shared__ double2 prow[2][NMAX];  // pivot rows of the Cholesky steps, by step parity
    if (tid < 2 * NMAX) prow[tid / NMAX][tid % NMAX] = make_double2(0.0, 0.0);  // columns past nB stay zero
    // R rows in pivot order over the B region: Rs[j][c] = R(j, position of column c)
    double2 (*const Rs)[NMAX] = reinterpret_cast<double2 (*)[NMAX]>(Bmem);
    // Every wave keeps the Schur complement's diagonal, lane c holding entry c, and updates it
    // from each pivot row, so each wave finds the next pivot by itself (the same one in every
    // wave) and the owners of that row publish it right after their update: one barrier per step.
    double dg = 0.0;
    unsigned long long usedmask = 0ull;
    // column of the largest remaining diagonal entry.  The key is the entry's high word (sign,
    // exponent and 20 mantissa bits, in the order of the values for non-negative ones) with its 6
    // lowest bits replaced by 63 - column, 0 for a used, padded or non-positive entry: entries
    // within ~2^-14 of each other count as equal and the lowest column wins.  With every key 0 it
    // returns 63, whose diagonal copy is then not positive, so the caller's stop test ends.
    auto next_pivot = [&]() -> int {
      unsigned key = 0u;
      if (lane < nB && !((usedmask >> lane) & 1ull) && dg > 0.0)
        key = ((unsigned)__double2hiint(dg) & ~63u) | (unsigned)(63 - lane);
      return 63 - (int)(wave_umax_uniform(key) & 63u);
    };
    int j = 0;
    if constexpr (NMAX == 64) {
      // D <= 32: S stays in the Gram tiles' registers and the rank-1 updates of four steps are
      // applied together, as one complex rank-4 product per tile on the matrix cores.  Until
      // then each pending row i is kept in registers twice, as rl[i] = R_i[lane] (any column by
      // readlane) and rc[q][i] = R_i at the lane's column of tile q; the owners of the next pivot
      // row apply the pending rows to it before publishing it.
      __shared__ double diag[NMAX];
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        int ti, tj;
        if (tile_ij(q, ti, tj) && ti == tj && (li & 3) == lk) {
          const int r = li >> 2;
          diag[16 * ti + li] = r == 0 ? sr[q][0] : r == 1 ? sr[q][1] : r == 2 ? sr[q][2] : sr[q][3];
        }
      }
      __syncthreads();
      if (lane < nB) dg = diag[lane];
      double2 rl[4], rc[TPW][4];
      auto publish_row = [&](int P, int np, int buf) {
        double2 rp[4];  // R_i[P] of the pending rows
#pragma unroll
        for (int i = 0; i < 4; ++i)
          rp[i] = i < np ? make_double2(readlane_d(rl[i].x, P), readlane_d(rl[i].y, P)) : make_double2(0.0, 0.0);
        const int rr = P & 15, r4 = rr >> 2;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
          int ti, tj;
          if (tile_ij(q, ti, tj) && ti == (P >> 4) && lk == (rr & 3)) {
            const int c = 16 * tj + li;
            double2 v = r4 == 0 ? make_double2(sr[q][0], si[q][0]) : r4 == 1 ? make_double2(sr[q][1], si[q][1])
                      : r4 == 2 ? make_double2(sr[q][2], si[q][2]) : make_double2(sr[q][3], si[q][3]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (i < np) v = csub(v, cmulc(rp[i], rc[q][i]));
            if (c < nB) prow[buf][c] = ((usedmask >> c) & 1ull) ? make_double2(0.0, 0.0) : v;
          }
        }
      };
      // the pivot, its diagonal value dP (lane copy) and 1 / sqrt(dP), ready before the barrier
      int P = next_pivot();
      double dP = readlane_d(dg, P);
      const double stop = dP * (64.0 * 2.220446049250313e-16);
      double rd = rsq_nr(dP);
      if (dP > stop) publish_row(P, 0, 0);
      __syncthreads();
      bool done = false;
      for (int jb = 0; !done; jb += 4) {
        if (jb > 0) {
          // S -= sum over the rows jb - 4 .. jb - 1 of conj(R_i[r]) R_i[c] (rows visible in LDS)
#pragma unroll
          for (int q = 0; q < TPW; ++q) {
            int ti, tj;
            if (tile_ij(q, ti, tj)) {
              const double2 a = Rs[jb - 4 + lk][16 * ti + li], b = Rs[jb - 4 + lk][16 * tj + li];
              sr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.x, b.x, sr[q], 0, 0, 0);
              sr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, sr[q], 0, 0, 0);
              si[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.x, b.y, si[q], 0, 0, 0);
              si[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, si[q], 0, 0, 0);
            }
          }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (j >= nB || !(dP > stop)) {  // the remaining Schur complement is rounding noise
            done = true;
            break;
          }
          const double2* pw = prow[j & 1];
          const double2 pv = pw[lane < NMAX ? lane : 0];  // first: the diagonal update waits only on it
          double2 pt[TPW];
#pragma unroll
          for (int q = 0; q < TPW; ++q) {
            int ti, tj;
            tile_ij(q, ti, tj);
            pt[q] = pw[(16 * tj + li) & (NMAX - 1)];
          }
          const double id = rd * rd;  // 1 / R(j, j)^2
          usedmask |= 1ull << P;
          dg = lane == P ? 0.0 : dg - cabs2(pv) * id;
          // row j of R, queued behind the reads (read after the barrier)
          rl[k] = cscale(pv, rd);
          if (tid == 0) colid[j] = P;
          if (tid < NMAX) Rs[j][tid] = tid >= nB ? make_double2(0.0, 0.0) : tid == P ? make_double2(dP * rd, 0.0) : rl[k];
          const int Pn = next_pivot();
          const double dPn = readlane_d(dg, Pn);
#pragma unroll
          for (int q = 0; q < TPW; ++q) rc[q][k] = cscale(pt[q], rd);
          ++j;
          if (j < nB && dPn > stop) publish_row(Pn, k + 1, j & 1);
          P = Pn;
          dP = dPn;
          rd = rsq_nr(dP);
          __syncthreads();
        }
      }
    } else {
      // D <= 16: the step is bound by its chain, not by issue: thread (br, bc) holds the E x E
      // block of rows br E.., columns bc E.. of S and applies every rank-1 update at once.
      constexpr int GB = NT == 256 ? 16 : 8;  // blocks per side
      constexpr int E = NMAX / GB;
      static_assert(GB * GB == NT && E * GB == NMAX, "Cholesky blocks");
      const int br = tid / GB, bc = tid - (tid / GB) * GB;
      __syncthreads();
      {
        double2 (*const Gs)[NMAX + 1] = reinterpret_cast<double2 (*)[NMAX + 1]>(Bmem);
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
          int ti, tj;
          if (tile_ij(q, ti, tj)) {
#pragma unroll
            for (int r = 0; r < 4; ++r) Gs[16 * ti + lk + 4 * r][16 * tj + li] = make_double2(sr[q][r], si[q][r]);
          }
        }
      }
      __syncthreads();
      double2 g[E][E];
      {
        double2 (*const Gs)[NMAX + 1] = reinterpret_cast<double2 (*)[NMAX + 1]>(Bmem);
#pragma unroll
        for (int a = 0; a < E; ++a)
#pragma unroll
          for (int b = 0; b < E; ++b) {
            const int r = br * E + a, c = bc * E + b;
            const double2 t = Gs[r][c];
            g[a][b] = (r < nB && c < nB) ? t : make_double2(0.0, 0.0);
          }
        if (lane < nB) dg = Gs[lane][lane].x;
      }
      auto publish_row = [&](int P, int buf) {
        if (br == P / E) {
#pragma unroll
          for (int a = 0; a < E; ++a)
            if (br * E + a == P)
#pragma unroll
              for (int b = 0; b < E; ++b)
                if (bc * E + b < nB) prow[buf][bc * E + b] = g[a][b];
        }
      };
      int P = next_pivot();
      double dP = readlane_d(dg, P);
      const double stop = dP * (64.0 * 2.220446049250313e-16);
      double rd = rsq_nr(dP);
      if (dP > stop) publish_row(P, 0);
      __syncthreads();
      for (; j < nB; ++j) {
        if (!(dP > stop)) break;  // the remaining Schur complement is rounding noise
        const double2* pw = prow[j & 1];
        // every LDS read of the step is issued here, the pivot row entry of the lane's column
        // first: the diagonal update and the next pivot wait only on it
        const double2 pv = pw[lane < NMAX ? lane : 0];
        double2 pr[E], pc[E];
#pragma unroll
        for (int a = 0; a < E; ++a) {
          pr[a] = pw[br * E + a];
          pc[a] = pw[bc * E + a];
        }
        const double id = rd * rd;  // 1 / R(j, j)^2
        usedmask |= 1ull << P;
        dg = lane == P ? 0.0 : dg - cabs2(pv) * id;
        // row j of R, queued behind the reads
        if (tid == 0) colid[j] = P;
        if (tid < nB) Rs[j][tid] = tid == P ? make_double2(dP * rd, 0.0) : cscale(pv, rd);
        const int Pn = next_pivot();
        const double dPn = readlane_d(dg, Pn);
        // S[r][c] -= conj(S[P][r]) S[P][c] / S[P][P] (S Hermitian).  The rows and columns of the
        // pivots already taken keep rounding residue instead of zeros: no entry of R, no diagonal
        // entry left in play and no update of an entry left in play reads them.
#pragma unroll
        for (int a = 0; a < E; ++a) {
          const double2 ps = cscale(pr[a], id);
#pragma unroll
          for (int b = 0; b < E; ++b) {
            g[a][b].x = fma(-ps.x, pc[b].x, fma(-ps.y, pc[b].y, g[a][b].x));
            g[a][b].y = fma(-ps.x, pc[b].y, fma(ps.y, pc[b].x, g[a][b].y));
          }
        }
        if (dPn > stop) publish_row(Pn, (j + 1) & 1);
        P = Pn;
        dP = dPn;
        rd = rsq_nr(dP);
        __syncthreads();
      }
    }
    // never-pivoted columns (zero Schur complement) follow in ascending order
    if (tid == 0)
      for (int c = 0, k = j; c < nB; ++c)
        if (!((usedmask >> c) & 1ull)) colid[k++] = c;
    __syncthreads();
    // B <- R^H on the leading nB x nB block: X[c][r] = conj(R(c, r)) = conj(Rs[c][colid[r]]),
    // c <= r, rows of R past the last pivot zero
    double2 xt[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int idx = tid + e * NT;
      const int c = idx / nB, rr = idx - (idx / nB) * nB;
      xt[e] = (idx < nB * nB && c <= rr && c < j) ? cconj(Rs[c][colid[rr]]) : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int idx = tid + e * NT;
      const int c = idx / nB, rr = idx - (idx / nB) * nB;
      if (idx < nB * nB) B[c][rr] = xt[e];
    }
    __syncthreads();
    mJ = nB;
  }

  const int np = nB + (nB & 1);
  const int npairs = np / 2;
  constexpr int LJ = 2 * NT / NMAX;  // lanes per column pair
  const int pair_id = tid / LJ;
  const int lane = tid - pair_id * LJ;
  // lane `lane` holds rows lane + LJ ((u + jsh) mod RPL); when several pairs share a 16-lane LDS
  // cycle (LJ < 16) they start on consecutive row blocks, so their accesses use disjoint banks
  constexpr int PW = LJ < 16 ? 16 / LJ : 1;  // pairs per 16-lane group
  static_assert((RPL & (RPL - 1)) == 0 && RPL >= PW, "Jacobi row blocks");
  const int jsh = pair_id & (PW - 1);
  auto jrow = [&](int u) { return lane + LJ * ((u + jsh) & (RPL - 1)); };
  const bool active = pair_id < npairs;
  const double tol2 = (2.220446049250313e-16 * (double)mJ) * (2.220446049250313e-16 * (double)mJ);
  int sweep = 0;
  bool converged = (nB < 2);
  if constexpr (PRE) {
    // Register-resident Jacobi (complex64 path, X = R^H: nB x nB).  The columns are padded to
    // 2^K >= nB and paired as {c, c ^ m} for m = 1 .. 2^K - 1, a complete sweep in which every
    // round is a perfect matching.  The rounds run in blocks of equal highest bit hb of m: inside
    // a block the column of the pair with bit hb clear stays in the registers of its lane group
    // g = c with bit hb deleted, and its partner (bit hb set) sits in group
    // g = (c ^ m) with bit hb deleted.  With the low bits m' = m - 2^hb taken in Gray-code
    // order, consecutive rounds differ in one bit b of m', so every moving column passes to
    // group g ^ 2^b: a lane permutation (lane ^ LJ 2^b) inside a wave, an LDS store, barrier and
    // load across waves.  Between blocks (and at the end of every sweep) all columns are written
    // to B and re-read under the next block's assignment.  The rotation arithmetic is that of
    // the LDS path below.
    constexpr int GW = 64 / LJ;  // lane groups per wave
    int K = 1;
    while ((1 << K) < nB) ++K;
    const bool gact = pair_id < (1 << (K - 1));
    auto ins = [](int g, int hb, int bit) { return ((g >> hb) << (hb + 1)) | (bit << hb) | (g & ((1 << hb) - 1)); };
    auto xrow = [&](int u) { return lane + LJ * u; };
    double2 xs[RPL], xm[RPL];  // stationary and moving column of the group
    double ns = 0.0, nm = 0.0;  // their tracked squared norms
    int cs_id = 0, cm_id = 0;   // their column indices
    auto load_col = [&](double2 (&x)[RPL], int c) {
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int rr = xrow(u);
        const double2 t = B[c][rr];
        x[u] = (gact && c < nB && rr < nB) ? t : make_double2(0.0, 0.0);
      }
    };
    auto store_col = [&](const double2 (&x)[RPL], int c, double n2) {
      if (gact && c < nB) {
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          const int rr = xrow(u);
          if (rr < nB) B[c][rr] = x[u];
        }
        if (lane == 0) nrm[c] = n2;
      }
    };
    auto col_norm = [&](const double2 (&x)[RPL]) {
      double s2 = 0.0;
#pragma unroll
      for (int u = 0; u < RPL; ++u) s2 += cabs2(x[u]);
      return group_sum_dpp(s2, LJ);
    };
    // per-sweep flags (any rotation, any rotation above the quiet level), three sets in
    // rotation so that a set is cleared neither while it is read nor after it is written
    __shared__ int sh_flag[3][2];
    if (tid < 6) sh_flag[tid >> 1][tid & 1] = 0;
    // the padding columns (ids nB .. 2^K - 1) and the ids of inactive groups are exactly zero:
    // their tracked norms are zero too (store_col never writes them), which keeps the rotation
    // scalars of every pair finite
    for (int c = nB + tid; c < NMAX; c += NT) nrm[c] = 0.0;
    bool rot = false, big = false;
    __syncthreads();
    const double floor2 = sh_floor * sh_floor;
    for (; sweep < st.max_sweeps && !converged; ++sweep) {
      for (int hb = 0; hb < K; ++hb) {
        cs_id = ins(pair_id, hb, 0);
        cm_id = ins(pair_id, hb, 1);
        load_col(xs, cs_id);
        load_col(xm, cm_id);
        if (hb == 0) {
          ns = col_norm(xs);
          nm = col_norm(xm);
        } else {
          ns = nrm[cs_id];
          nm = nrm[cm_id];
        }
        const int nt = 1 << hb;
        // the moving column passes to group pair_id ^ 2^bb (lane ^ LJ 2^bb inside a wave)
        auto move_intra = [&](auto tag) {
          constexpr int OFF = decltype(tag)::value;
#pragma unroll
          for (int u = 0; u < RPL; ++u) lane_xor_pair<OFF>(xm[u].x, xm[u].y);
          nm = lane_xor<OFF>(nm);
        };
        auto move_off = [&](int off) {
          if (off == 4) move_intra(std::integral_constant<int, 4>());
          else if (off == 8) move_intra(std::integral_constant<int, 8>());
          else if (off == 16) move_intra(std::integral_constant<int, 16>());
          else move_intra(std::integral_constant<int, 32>());
        };
        // one round: the rotation of the group's pair (stationary xs, moving xm).  Branch-free:
        // a pair that is not rotated takes c = 1, s = 0 (f = 0), which leaves both columns and
        // norms bit for bit.  Padding columns are exactly zero, so their pairs have g = 0 and are
        // never rotated; h is kept away from zero so that every pair's scalars stay finite.
        auto round = [&]() {
          double2 g = cmulc(xs[0], xm[0]);
#pragma unroll
          for (int u = 1; u < RPL; ++u) g = cadd(g, cmulc(xs[u], xm[u]));
          double gr = g.x, gi = g.y;
          group_sum2_dpp(gr, gi, LJ);
          const double al = ns, be = nm;
          const double g2 = gr * gr + gi * gi;
          const double ab = al * be;
          const bool ok = (g2 > tol2 * ab) & (g2 > floor2);
          const double d = be - al;
          const double h2 = fmax(d * d + 4.0 * g2, 1e-300);
          const double rh = rsq_nr1(h2);  // 1 / h
          const double x = 0.5 + 0.5 * fabs(d) * rh;
          const double rc = rsq_nr1(x);   // 1 / c
          const double f = ok ? copysign(rh, d) * rc : 0.0;
          const double cs = ok ? x * rc : 1.0;
          const double2 sph = make_double2(gr * f, gi * f);  // s e^{i phi}
          const double tg = g2 * f * rc;                      // t |g|
#pragma unroll
          for (int u = 0; u < RPL; ++u) {
            const double2 bp = xs[u], bq = xm[u];
            xs[u] = csub(cscale(bp, cs), cmulc(sph, bq));
            xm[u] = cadd(cmul(sph, bp), cscale(bq, cs));
          }
          ns = al - tg;
          nm = be + tg;
          rot |= ok;
          big |= ok & (g2 > kJacobiQuietC64 * ab);
        };
        // the moving column of this group in round t of the block
        auto mid = [&](int t) { return ins(pair_id ^ (t ^ (t >> 1)), hb, 1); };
        // groups of up to 8 rounds (4 when a lane holds 8 or more rows: straight-line groups
        // that long take the compiler many minutes for little gain)
        constexpr int UN = RPL >= 8 ? (GW < 4 ? GW : 4) : (GW < 8 ? GW : 8);
        if (nt < UN) {
          // short block (2^hb rounds, all moves inside a wave)
          for (int t = 0; t < nt; ++t) {
            round();
            if (t + 1 < nt) move_off(LJ << __builtin_ctz(t + 1));
          }
        } else {
          // rounds in groups of UN (nt is a multiple of UN): inside a group the bit that changes
          // between consecutive rounds, ctz(k + 1), is a compile-time constant and every move is
          // unconditional straight-line code; only the move after a group can cross waves
          for (int t0 = 0; t0 < nt; t0 += UN) {
#pragma unroll
            for (int k = 0; k < UN; ++k) {
              round();
              const int t = t0 + k;
              if (k + 1 < UN) {
                move_off(LJ << __builtin_ctz(k + 1));  // folds to one straight-line move
              } else if (t + 1 < nt) {
                const int bb = __builtin_ctz(t + 1);
                if ((1 << bb) < GW) {
                  move_off(LJ << bb);
                } else {
                  store_col(xm, mid(t), nm);
                  __syncthreads();
                  load_col(xm, mid(t + 1));
                  nm = nrm[mid(t + 1)];
                }
              }
            }
          }
        }
        cm_id = mid(nt - 1);
        // end of the block: every column back to B (with its tracked norm)
        store_col(xs, cs_id, ns);
        store_col(xm, cm_id, nm);
        if (hb + 1 == K) {
          if (rot && lane == 0) sh_flag[sweep % 3][0] = 1;
          if (big && lane == 0) sh_flag[sweep % 3][1] = 1;
          if (tid < 2) sh_flag[(sweep + 1) % 3][tid] = 0;
          rot = false;
          big = false;
        }
        __syncthreads();
      }
      // complex64 path: a sweep whose rotations all had |g|^2 <= 1e-12 al be ends the iteration
      converged = (sh_flag[sweep % 3][0] == 0) || (sh_flag[sweep % 3][1] == 0);
    }
  } else {
  for (; sweep < st.max_sweeps && !converged; ++sweep) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = 2 * pair_id + h;
      double s2 = 0.0;
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int rr = jrow(u);
        const double2 t = B[c][rr];
        if (c < nB && rr < mJ) s2 += cabs2(t);
      }
      s2 = group_sum_dpp(s2, LJ);
      if (lane == 0 && c < nB) nrm[c] = s2;
    }
    if (tid == 0) {
      sh_rot = 0;
      sh_big = 0;
    }
    __syncthreads();
    const double floor2 = sh_floor * sh_floor;
    // circle-method tournament: slot 0 fixed, the others advance by one each round
    int pa = pair_id;
    int pb = np - 1 - pair_id;
    for (int round = 0; round < np - 1; ++round) {
      const bool work = active && (pa < nB) && (pb < nB);
      const int p = work ? (pa < pb ? pa : pb) : 0;
      const int q = work ? (pa < pb ? pb : pa) : 0;
      // every load of the round is issued before the first use
      double2 bp[RPL], bq[RPL];
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const int rr = jrow(u);
        const double2 a = B[p][rr], b = B[q][rr];
        const bool ok = work && rr < mJ;
        bp[u] = ok ? a : make_double2(0.0, 0.0);
        bq[u] = ok ? b : make_double2(0.0, 0.0);
      }
      const double al = nrm[p], be = nrm[q];
      double gr = 0.0, gi = 0.0;
#pragma unroll
      for (int u = 0; u < RPL; ++u) {
        const double2 gg = cmulc(bp[u], bq[u]);
        gr += gg.x;
        gi += gg.y;
      }
      asm volatile("" ::"v"(al), "v"(be));  // keeps the norm loads beside the row loads
      group_sum2_dpp(gr, gi, LJ);
      if (work) {
        const double g2 = gr * gr + gi * gi;
        if (g2 > tol2 * al * be && g2 > floor2) {
          double2 wp[ACC ? RPL : 1], wq[ACC ? RPL : 1];
          if (ACC) {
#pragma unroll
            for (int u = 0; u < RPL; ++u) {
              const int rr = jrow(u);
              wp[u] = W[p][rr];
              wq[u] = W[q][rr];
            }
          }
          // The rotation of smaller angle (|theta| <= pi/4) with tan 2 theta = 2|g| / (be - al):
          // h = (d^2 + 4|g|^2)^1/2, d = be - al, x = cos^2 theta = (1 + |d| / h) / 2, and
          // c = x^1/2, s e^{i phi} = sign(d) g / (h x^1/2), so c^2 + |s|^2 = 1 exactly in exact
          // arithmetic and |g| itself is never formed.  Two reciprocal square roots (two Newton
          // steps each; one on the complex64 path) are the whole dependent chain.
          const double d = be - al;
          const double h2 = d * d + 4.0 * g2;
          const double rh = PRE ? rsq_nr1(h2) : rsq_nr(h2);  // 1 / h
          const double x = 0.5 + 0.5 * fabs(d) * rh;
          const double rc = PRE ? rsq_nr1(x) : rsq_nr(x);    // 1 / c
          const double cs = x * rc;
          const double f = (d < 0.0 ? -rh : rh) * rc;
          const double2 sph = make_double2(gr * f, gi * f);  // s e^{i phi}
          const double tg = g2 * f * rc;                      // t |g| = sign(d) |g|^2 / (h c^2)
          // b_p' = c b_p - s e^{-i phi} b_q ;  b_q' = s e^{i phi} b_p + c b_q
#pragma unroll
          for (int u = 0; u < RPL; ++u) {
            const int rr = jrow(u);
            if (rr < mJ) {
              B[p][rr] = csub(cscale(bp[u], cs), cmulc(sph, bq[u]));
              B[q][rr] = cadd(cmul(sph, bp[u]), cscale(bq[u], cs));
            }
          }
          if (ACC) {
#pragma unroll
            for (int u = 0; u < RPL; ++u) {
              const int rr = jrow(u);
              if (rr < nB) {
                W[p][rr] = csub(cscale(wp[u], cs), cmulc(sph, wq[u]));
                W[q][rr] = cadd(cmul(sph, wp[u]), cscale(wq[u], cs));
              }
            }
          }
          if (lane == 0) {
            nrm[p] = al - tg;
            nrm[q] = be + tg;
            sh_rot = 1;
            if (g2 > kJacobiQuiet * al * be) sh_big = 1;
          }
        }
      }
      if (pair_id != 0) pa = (pa == np - 1) ? 1 : pa + 1;
      pb = (pb == np - 1) ? 1 : pb + 1;
      __syncthreads();
    }
    // complex64 path: a sweep whose rotations all had |g|^2 <= 1e-12 al be leaves
    // off-diagonal terms of second order, O(n 1e-12) relative, far below the complex64 storage
    // rounding, so it ends the iteration without a rotation-free check sweep
    converged = (sh_rot == 0) || (PRE && sh_big == 0);
    __syncthreads();
  }
  }
  if (tid == 0) {
    atomicAdd(reinterpret_cast<unsigned long long*>(st.stats) + 0, (unsigned long long)sweep);
    atomicAdd(reinterpret_cast<unsigned long long*>(st.stats) + 1, 1ull);
    atomicMax(reinterpret_cast<unsigned long long*>(st.stats) + 2, (unsigned long long)sweep);
    if (!converged) {
      atomicAdd(reinterpret_cast<unsigned long long*>(st.stats) + 3, 1ull);
      flag_status(st.status, kStatusNoConverge);
    }
  }

  // singular values (column norms, two columns per pair group), stable descending order
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = 2 * pair_id + h;
    double s2 = 0.0;
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int rr = jrow(u);
      const double2 t = B[c][rr];
      if (c < nB && rr < mJ) s2 += cabs2(t);
    }
    s2 = group_sum_dpp(s2, LJ);
    if (lane == 0 && c < nB) sig[c] = sqrt(s2);
  }
  __syncthreads();
  for (int c = tid; c < nB; c += NT) {
    const double sv = sig[c];
    int rank = 0;
    for (int d = 0; d < nB; ++d) {
      const double sd = sig[d];
      rank += (sd > sv) || (sd == sv && d < c);
    }
    perm[rank] = c;
  }
  __syncthreads();
  // truncation (one wave; nB <= 64): chi = #{sigma > trunc_rel sigma_0} capped at D (at least
  // 1), and the norm of the kept values for lambda_e
  if (tid < 64) {
    const double smax = sig[perm[0]];
    const int keep = __popcll(__ballot(tid < nB && sig[tid] > st.trunc_rel * smax));
    int chi = keep < D ? keep : D;
    if (chi < 1) chi = 1;
    const double sk = tid < chi ? sig[perm[tid]] : 0.0;
    const double nr = sqrt(group_sum_dpp(sk * sk, 64));
    if (tid == 0) {
      if (!(smax > 0.0)) flag_status(st.status, kStatusZeroTheta);
      if (!isfinite(nr)) flag_status(st.status, kStatusNonFinite);
      sh_chi = chi;
      sh_norm = nr;
      st.meta[slot].de_old = de;
      st.meta[slot].chi_new = chi;
      st.chi[e] = chi;
    }
  }
  __syncthreads();
  const int chi = sh_chi;
  for (int k = tid; k < D; k += NT) lam_e[k] = k < chi ? sig[perm[k]] / sh_norm : 0.0;
  if (BWD) {
    // every singular triplet: U [m0 x r], V [n0 x r], S [r], r = nB, row stride 2D; vectors
    // with sigma <= 1e-13 sigma_0 are set to zero (the null space)
    const int ld = 2 * D;
    double2* Ug = st.bU + (int64_t)slot * ld * ld;
    double2* Vg = st.bV + (int64_t)slot * ld * ld;
    const double smax = sig[perm[0]];
    for (int k = tid; k < nB; k += NT) st.bS[(int64_t)slot * ld + k] = sig[perm[k]];
    if (ACC) {
      for (int idx = tid; idx < mB * nB; idx += NT) {
        const int rr = idx / nB, k = idx - (idx / nB) * nB;
        const double sv = sig[perm[k]];
        const double2 bv = sv > 1e-13 * smax ? cscale(B[perm[k]][rr], 1.0 / sv) : make_double2(0.0, 0.0);
        (trans ? Vg : Ug)[rr * ld + k] = bv;
      }
      for (int idx = tid; idx < nB * nB; idx += NT) {
        const int rr = idx / nB, k = idx - (idx / nB) * nB;
        (trans ? Ug : Vg)[rr * ld + k] = W[perm[k]][rr];
      }
    } else {
      // preconditioned path: the Jacobi side is B's right singular vectors (rows permuted by the
      // pivoting), i.e. V of Theta' when B = Theta', U when B = Theta'^H
      for (int idx = tid; idx < nB * nB; idx += NT) {
        const int rr = idx / nB, k = idx - (idx / nB) * nB;
        const double sv = sig[perm[k]];
        const double2 bv = sv > 1e-13 * smax ? cscale(B[perm[k]][rr], 1.0 / sv) : make_double2(0.0, 0.0);
        (trans ? Ug : Vg)[colid[rr] * ld + k] = bv;
      }
    }
  }

  CT* T = reinterpret_cast<CT*>(st.tbuf);
  CT* const Ti0 = T + rbuf_off(st, slot, 0, 0);
  CT* const Ti1 = T + rbuf_off(st, slot, 0, 1);
  CT* const Tj0 = T + rbuf_off(st, slot, 1, 0);
  CT* const Tj1 = T + rbuf_off(st, slot, 1, 1);
  // zero columns k' >= chi of every T (rows k < de)
  for (int idx = tid; idx < 4 * de * (D - chi); idx += NT) {
    const int w = idx / (de * (D - chi));
    const int rem = idx - w * de * (D - chi);
    const int k = rem / (D - chi), kp = chi + rem - (rem / (D - chi)) * (D - chi);
    if (BWD) st.t64[rbuf_off(st, slot, w >> 1, w & 1) + k * D + kp] = make_double2(0.0, 0.0);
    T[rbuf_off(st, slot, w >> 1, w & 1) + k * D + kp] = from_d2<CT>(make_double2(0.0, 0.0));
  }
  const double2 g00 = gate_phase(ip, 0, 0), g01 = gate_phase(ip, 0, 1);
  const double2 g10 = gate_phase(ip, 1, 0), g11 = gate_phase(ip, 1, 1);
  // T_w[k][k'] (w = 0, 1: end i slices; 2, 3: end j slices), float64 in the reverse sweep
  auto putT = [&](int w, int k, int kp, double2 v) {
    if (BWD) st.t64[rbuf_off(st, slot, w >> 1, w & 1) + k * D + kp] = v;
    T[rbuf_off(st, slot, w >> 1, w & 1) + k * D + kp] = from_d2<CT>(v);
  };

  if (ACC) {
    // both vector sets are available: U / V from B and W, straight into the arena
    double2 uv[2 * RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int idx = tid + u * NT;
      uv[u] = make_double2(0.0, 0.0);
      uv[RPT + u] = make_double2(0.0, 0.0);
      if (idx < mB * chi) {
        const int rr = idx / chi, kp = idx - (idx / chi) * chi;
        uv[u] = cscale(B[perm[kp]][rr], 1.0 / sig[perm[kp]]);
      }
      if (idx < nB * chi) {
        const int rr = idx / chi, kp = idx - (idx / chi) * chi;
        uv[RPT + u] = W[perm[kp]][rr];
      }
    }
    __syncthreads();
    double2* Ul = A0;  // U [(s,a)][k'], row stride DS
    double2* Vl = Wmem;  // V [(t,b)][k'], row stride DS
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int idx = tid + u * NT;
      if (idx < mB * chi) {
        const int rr = idx / chi, kp = idx - (idx / chi) * chi;
        (trans ? Vl : Ul)[rr * DS + kp] = uv[u];
      }
      if (idx < nB * chi) {
        const int rr = idx / chi, kp = idx - (idx / chi) * chi;
        (trans ? Ul : Vl)[rr * DS + kp] = uv[RPT + u];
      }
    }
    __syncthreads();
    stage_r(A1, 0, ri);
    stage_r(Wmem + 2 * DM * DS, 1, rj);
    __syncthreads();
    const double2* RIl = A1;
    const double2* RJl = Wmem + 2 * DM * DS;
    for (int idx = tid; idx < de * chi; idx += NT) {
      const int k = idx / chi, kp = idx - (idx / chi) * chi;
      double2 x0 = make_double2(0.0, 0.0), x1 = x0, y0 = x0, y1 = x0;
      for (int b = 0; b < rj; ++b) {
        x0 = cadd(x0, cmul(RJl[b * DS + k], Vl[b * DS + kp]));
        x1 = cadd(x1, cmul(RJl[DM * DS + b * DS + k], Vl[(rj + b) * DS + kp]));
      }
      for (int a2 = 0; a2 < ri; ++a2) {
        y0 = cadd(y0, cmulc(Ul[a2 * DS + kp], RIl[a2 * DS + k]));
        y1 = cadd(y1, cmulc(Ul[(ri + a2) * DS + kp], RIl[DM * DS + a2 * DS + k]));
      }
      const double f = lam_old[k] / sig[perm[kp]];
      const double2 ti0 = cscale(cadd(cmul(g00, x0), cmul(g01, x1)), f);
      const double2 ti1 = cscale(cadd(cmul(g10, x0), cmul(g11, x1)), f);
      const double2 tj0 = cscale(cadd(cmul(g00, y0), cmul(g10, y1)), f);
      const double2 tj1 = cscale(cadd(cmul(g01, y0), cmul(g11, y1)), f);
      if (BWD) {
        double2* T64 = st.t64 + rbuf_off(st, slot, 0, 0);
        T64[0 * D * D + k * D + kp] = ti0;
        T64[1 * D * D + k * D + kp] = ti1;
        T64[2 * D * D + k * D + kp] = tj0;
        T64[3 * D * D + k * D + kp] = tj1;
      }
      {
        Ti0[k * D + kp] = from_d2<CT>(ti0);
        Ti1[k * D + kp] = from_d2<CT>(ti1);
        Tj0[k * D + kp] = from_d2<CT>(tj0);
        Tj1[k * D + kp] = from_d2<CT>(tj1);
      }
    }
    return;
  }

  // complex64 path: the Jacobi side from B, the other side through small products with the R
  // factors.  After preconditioning the Jacobi side is B's right singular vectors: V of Theta'
  // when B = Theta', U of Theta' when B = Theta'^H, so the orientation below is flipped.
  const bool vside = !trans;  // the Jacobi side holds V (rows (t,b)) rather than U (rows (s,a))
  {
    double2 v[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int idx = tid + u * NT;
      v[u] = make_double2(0.0, 0.0);
      if (idx < nB * chi) {
        const int rr = idx / chi, kp = idx - (idx / chi) * chi;
        v[u] = cscale(B[perm[kp]][rr], 1.0 / sig[perm[kp]]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int idx = tid + u * NT;
      if (idx < nB * chi) {
        const int rr = idx / chi, kp = idx - (idx / chi) * chi;
        A0[colid[rr] * DS + kp] = v[u];  // V [(t,b)][k'] or U [(s,a)][k']
      }
    }
    stage_r(A1, vside ? 1 : 0, vside ? rj : ri);
    __syncthreads();
  }
  if constexpr (NMAX == 64) {
    // The three small products below run on the FP64 matrix cores as 16 x 16 output tiles, one
    // tile position per wave with both slices (s or t = 0, 1) in it (at most four positions:
    // D <= 32); results stay in registers across the barrier that frees the LDS they overwrite.
    static_assert(NMAX <= 32 || NT >= 256, "one tile position per wave");
    const int wv = tid >> 6, li = tid & 15, lk = (tid & 63) >> 4;
    auto tile_of = [&](int rows, int& ti, int& tj) {
      const int tn = (chi + 15) >> 4;
      ti = wv / tn;
      tj = wv - ti * tn;
      return wv < ((rows + 15) >> 4) * tn;
    };
    cgemm_d4 ar[2], ai[2];
    int ti = 0, tj = 0;
    if (!vside) {
      // Y_s = R_i^(s)H U_s;  T_j^(t) = lambda/sigma sum_s g(s,t) conj(Y_s);  Z_t = sum_s conj(g(s,t)) Y_s
      const bool tw = tile_of(de, ti, tj);
      if (tw) {
  #pragma unroll
        for (int h = 0; h < 2; ++h) {
          auto fa = [&](int k, int a) -> double2 {
            return (k < de && a < ri) ? cconj(A1[h * DM * DS + a * DS + k]) : make_double2(0.0, 0.0);
          };
          auto fb = [&](int a, int kp) -> double2 {
            return (a < ri && kp < chi) ? A0[(h * ri + a) * DS + kp] : make_double2(0.0, 0.0);
          };
          cgemm_tile(16 * ti, 16 * tj, ri, fa, fb, ar[h], ai[h]);
        }
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = 16 * ti + lk + 4 * r, kp = 16 * tj + li;
          const double2 y0 = make_double2(ar[0][r], ai[0][r]), y1 = make_double2(ar[1][r], ai[1][r]);
          if (k < de && kp < chi) {
            const double f = lam_old[k] / sig[perm[kp]];
            putT(2, k, kp, cscale(cadd(cmulc(y0, g00), cmulc(y1, g10)), f));
            putT(3, k, kp, cscale(cadd(cmulc(y0, g01), cmulc(y1, g11)), f));
          }
          const double2 z0 = cadd(cmulc(g00, y0), cmulc(g10, y1)), z1 = cadd(cmulc(g01, y0), cmulc(g11, y1));
          ar[0][r] = z0.x;
          ai[0][r] = z0.y;
          ar[1][r] = z1.x;
          ai[1][r] = z1.y;
        }
      }
      __syncthreads();
      if (tw) {
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = 16 * ti + lk + 4 * r, kp = 16 * tj + li;
          if (k < de && kp < chi) {
            A0[k * DS + kp] = make_double2(ar[0][r], ai[0][r]);
            A0[DM * DS + k * DS + kp] = make_double2(ar[1][r], ai[1][r]);
          }
        }
      }
      stage_r(A1, 1, rj);
      __syncthreads();
      // V_t[b][k'] = 1/sigma sum_k conj(R_j^(t)[b,k]) lambda_k Z_t[k][k']
      const bool tv = tile_of(rj, ti, tj);
      if (tv) {
  #pragma unroll
        for (int h = 0; h < 2; ++h) {
          auto fa = [&](int b, int k) -> double2 {
            return (b < rj && k < de) ? cscale(cconj(A1[h * DM * DS + b * DS + k]), lam_old[k]) : make_double2(0.0, 0.0);
          };
          auto fb = [&](int k, int kp) -> double2 {
            return (k < de && kp < chi) ? A0[h * DM * DS + k * DS + kp] : make_double2(0.0, 0.0);
          };
          cgemm_tile(16 * ti, 16 * tj, de, fa, fb, ar[h], ai[h]);
        }
      }
      __syncthreads();
      if (tv) {
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int b = 16 * ti + lk + 4 * r, kp = 16 * tj + li;
          if (b < rj && kp < chi) {
            const double is = 1.0 / sig[perm[kp]];
            A0[b * DS + kp] = cscale(make_double2(ar[0][r], ai[0][r]), is);
            A0[(rj + b) * DS + kp] = cscale(make_double2(ar[1][r], ai[1][r]), is);
          }
        }
      }
      __syncthreads();
      // T_i^(s) = lambda/sigma sum_t g(s,t) R_j^(t)T V_t
      if (tile_of(de, ti, tj)) {
  #pragma unroll
        for (int h = 0; h < 2; ++h) {
          auto fa = [&](int k, int b) -> double2 {
            return (k < de && b < rj) ? A1[h * DM * DS + b * DS + k] : make_double2(0.0, 0.0);
          };
          auto fb = [&](int b, int kp) -> double2 {
            return (b < rj && kp < chi) ? A0[(h * rj + b) * DS + kp] : make_double2(0.0, 0.0);
          };
          cgemm_tile(16 * ti, 16 * tj, rj, fa, fb, ar[h], ai[h]);
        }
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = 16 * ti + lk + 4 * r, kp = 16 * tj + li;
          if (k < de && kp < chi) {
            const double2 x0 = make_double2(ar[0][r], ai[0][r]), x1 = make_double2(ar[1][r], ai[1][r]);
            const double f = lam_old[k] / sig[perm[kp]];
            putT(0, k, kp, cscale(cadd(cmul(g00, x0), cmul(g01, x1)), f));
            putT(1, k, kp, cscale(cadd(cmul(g10, x0), cmul(g11, x1)), f));
          }
        }
      }
    } else {
      // X_t = R_j^(t)T V_t;  T_i^(s) = lambda/sigma sum_t g(s,t) X_t;  P_s = lambda sum_t g(s,t) X_t
      const bool tw = tile_of(de, ti, tj);
      if (tw) {
  #pragma unroll
        for (int h = 0; h < 2; ++h) {
          auto fa = [&](int k, int b) -> double2 {
            return (k < de && b < rj) ? A1[h * DM * DS + b * DS + k] : make_double2(0.0, 0.0);
          };
          auto fb = [&](int b, int kp) -> double2 {
            return (b < rj && kp < chi) ? A0[(h * rj + b) * DS + kp] : make_double2(0.0, 0.0);
          };
          cgemm_tile(16 * ti, 16 * tj, rj, fa, fb, ar[h], ai[h]);
        }
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = 16 * ti + lk + 4 * r, kp = 16 * tj + li;
          const double2 x0 = make_double2(ar[0][r], ai[0][r]), x1 = make_double2(ar[1][r], ai[1][r]);
          const double lk_ = k < de ? lam_old[k] : 0.0;
          const double2 p0 = cscale(cadd(cmul(g00, x0), cmul(g01, x1)), lk_);
          const double2 p1 = cscale(cadd(cmul(g10, x0), cmul(g11, x1)), lk_);
          if (k < de && kp < chi) {
            const double is = 1.0 / sig[perm[kp]];
            putT(0, k, kp, cscale(p0, is));
            putT(1, k, kp, cscale(p1, is));
          }
          ar[0][r] = p0.x;
          ai[0][r] = p0.y;
          ar[1][r] = p1.x;
          ai[1][r] = p1.y;
        }
      }
      __syncthreads();
      if (tw) {
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = 16 * ti + lk + 4 * r, kp = 16 * tj + li;
          if (k < de && kp < chi) {
            A0[k * DS + kp] = make_double2(ar[0][r], ai[0][r]);
            A0[DM * DS + k * DS + kp] = make_double2(ar[1][r], ai[1][r]);
          }
        }
      }
      stage_r(A1, 0, ri);
      __syncthreads();
      // U_s[a][k'] = 1/sigma sum_k R_i^(s)[a,k] P_s[k][k']
      const bool tu = tile_of(ri, ti, tj);
      if (tu) {
  #pragma unroll
        for (int h = 0; h < 2; ++h) {
          auto fa = [&](int a, int k) -> double2 {
            return (a < ri && k < de) ? A1[h * DM * DS + a * DS + k] : make_double2(0.0, 0.0);
          };
          auto fb = [&](int k, int kp) -> double2 {
            return (k < de && kp < chi) ? A0[h * DM * DS + k * DS + kp] : make_double2(0.0, 0.0);
          };
          cgemm_tile(16 * ti, 16 * tj, de, fa, fb, ar[h], ai[h]);
        }
      }
      __syncthreads();
      if (tu) {
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = 16 * ti + lk + 4 * r, kp = 16 * tj + li;
          if (a < ri && kp < chi) {
            const double is = 1.0 / sig[perm[kp]];
            A0[a * DS + kp] = cscale(make_double2(ar[0][r], ai[0][r]), is);
            A0[(ri + a) * DS + kp] = cscale(make_double2(ar[1][r], ai[1][r]), is);
          }
        }
      }
      __syncthreads();
      // T_j^(t) = lambda/sigma sum_s g(s,t) R_i^(s)T conj(U_s)
      if (tile_of(de, ti, tj)) {
  #pragma unroll
        for (int h = 0; h < 2; ++h) {
          auto fa = [&](int k, int a) -> double2 {
            return (k < de && a < ri) ? A1[h * DM * DS + a * DS + k] : make_double2(0.0, 0.0);
          };
          auto fb = [&](int a, int kp) -> double2 {
            return (a < ri && kp < chi) ? cconj(A0[(h * ri + a) * DS + kp]) : make_double2(0.0, 0.0);
          };
          cgemm_tile(16 * ti, 16 * tj, ri, fa, fb, ar[h], ai[h]);
        }
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = 16 * ti + lk + 4 * r, kp = 16 * tj + li;
          if (k < de && kp < chi) {
            const double2 y0 = make_double2(ar[0][r], ai[0][r]), y1 = make_double2(ar[1][r], ai[1][r]);
            const double f = lam_old[k] / sig[perm[kp]];
            putT(2, k, kp, cscale(cadd(cmul(g00, y0), cmul(g10, y1)), f));
            putT(3, k, kp, cscale(cadd(cmul(g01, y0), cmul(g11, y1)), f));
          }
        }
      }
    }
  } else {
    // D <= 16: every product is one 16 x 16 tile per physical slice, so wave h (h = 0, 1) takes
    // slice h on the matrix cores (one wave takes both when the workgroup has one); the two
    // slices meet in LDS, where every thread combines them for its (k, k') entry.
    constexpr int NW = NT / 64;
    static_assert(DM <= 16, "one tile per slice");
    const int wv = tid >> 6, li = tid & 15, lk = (tid & 63) >> 4;
    __shared__ double2 Xs[2][16][17];
    cgemm_d4 cr, ci;
    if (!vside) {
      // Y_s = R_i^(s)H U_s;  T_j^(t) = lambda/sigma sum_s g(s,t) conj(Y_s);  Z_t = sum_s conj(g(s,t)) Y_s
      for (int h = wv; h < 2; h += NW) {
        auto fa = [&](int k, int a) -> double2 {
          return (k < de && a < ri) ? cconj(A1[h * DM * DS + a * DS + k]) : make_double2(0.0, 0.0);
        };
        auto fb = [&](int a, int kp) -> double2 {
          return (a < ri && kp < chi) ? A0[(h * ri + a) * DS + kp] : make_double2(0.0, 0.0);
        };
        cgemm_tile(0, 0, ri, fa, fb, cr, ci);
#pragma unroll
        for (int r = 0; r < 4; ++r) Xs[h][lk + 4 * r][li] = make_double2(cr[r], ci[r]);
      }
      __syncthreads();
      for (int idx = tid; idx < 256; idx += NT) {
        const int k = idx >> 4, kp = idx & 15;
        if (k < de && kp < chi) {
          const double2 y0 = Xs[0][k][kp], y1 = Xs[1][k][kp];
          const double f = lam_old[k] / sig[perm[kp]];
          putT(2, k, kp, cscale(cadd(cmulc(y0, g00), cmulc(y1, g10)), f));
          putT(3, k, kp, cscale(cadd(cmulc(y0, g01), cmulc(y1, g11)), f));
          A0[k * DS + kp] = cadd(cmulc(g00, y0), cmulc(g10, y1));
          A0[DM * DS + k * DS + kp] = cadd(cmulc(g01, y0), cmulc(g11, y1));
        }
      }
      stage_r(A1, 1, rj);
      __syncthreads();
      // V_t[b][k'] = 1/sigma sum_k conj(R_j^(t)[b,k]) lambda_k Z_t[k][k'], then
      // X_t = R_j^(t)T V_t (each wave on its own slice: no barrier between the two)
      for (int h = wv; h < 2; h += NW) {
        auto fa = [&](int b, int k) -> double2 {
          return (b < rj && k < de) ? cscale(cconj(A1[h * DM * DS + b * DS + k]), lam_old[k]) : make_double2(0.0, 0.0);
        };
        auto fb = [&](int k, int kp) -> double2 {
          return (k < de && kp < chi) ? A0[h * DM * DS + k * DS + kp] : make_double2(0.0, 0.0);
        };
        cgemm_tile(0, 0, de, fa, fb, cr, ci);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double is = li < chi ? 1.0 / sig[perm[li]] : 0.0;
          Xs[h][lk + 4 * r][li] = cscale(make_double2(cr[r], ci[r]), is);
        }
        wave_lds_sync();
        auto fc = [&](int k, int b) -> double2 {
          return (k < de && b < rj) ? A1[h * DM * DS + b * DS + k] : make_double2(0.0, 0.0);
        };
        auto fd = [&](int b, int kp) -> double2 { return b < rj ? Xs[h][b][kp] : make_double2(0.0, 0.0); };
        cgemm_tile(0, 0, rj, fc, fd, cr, ci);
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r) Xs[h][lk + 4 * r][li] = make_double2(cr[r], ci[r]);
      }
      __syncthreads();
      // T_i^(s) = lambda/sigma sum_t g(s,t) X_t
      for (int idx = tid; idx < 256; idx += NT) {
        const int k = idx >> 4, kp = idx & 15;
        if (k < de && kp < chi) {
          const double2 x0 = Xs[0][k][kp], x1 = Xs[1][k][kp];
          const double f = lam_old[k] / sig[perm[kp]];
          putT(0, k, kp, cscale(cadd(cmul(g00, x0), cmul(g01, x1)), f));
          putT(1, k, kp, cscale(cadd(cmul(g10, x0), cmul(g11, x1)), f));
        }
      }
    } else {
      // X_t = R_j^(t)T V_t;  T_i^(s) = lambda/sigma sum_t g(s,t) X_t;  P_s = lambda sum_t g(s,t) X_t
      for (int h = wv; h < 2; h += NW) {
        auto fa = [&](int k, int b) -> double2 {
          return (k < de && b < rj) ? A1[h * DM * DS + b * DS + k] : make_double2(0.0, 0.0);
        };
        auto fb = [&](int b, int kp) -> double2 {
          return (b < rj && kp < chi) ? A0[(h * rj + b) * DS + kp] : make_double2(0.0, 0.0);
        };
        cgemm_tile(0, 0, rj, fa, fb, cr, ci);
#pragma unroll
        for (int r = 0; r < 4; ++r) Xs[h][lk + 4 * r][li] = make_double2(cr[r], ci[r]);
      }
      __syncthreads();
      for (int idx = tid; idx < 256; idx += NT) {
        const int k = idx >> 4, kp = idx & 15;
        if (k < de && kp < chi) {
          const double2 x0 = Xs[0][k][kp], x1 = Xs[1][k][kp];
          const double2 p0 = cscale(cadd(cmul(g00, x0), cmul(g01, x1)), lam_old[k]);
          const double2 p1 = cscale(cadd(cmul(g10, x0), cmul(g11, x1)), lam_old[k]);
          const double is = 1.0 / sig[perm[kp]];
          putT(0, k, kp, cscale(p0, is));
          putT(1, k, kp, cscale(p1, is));
          A0[k * DS + kp] = p0;
          A0[DM * DS + k * DS + kp] = p1;
        }
      }
      stage_r(A1, 0, ri);
      __syncthreads();
      // U_s[a][k'] = 1/sigma sum_k R_i^(s)[a,k] P_s[k][k'], then Y_s = R_i^(s)T conj(U_s)
      for (int h = wv; h < 2; h += NW) {
        auto fa = [&](int a, int k) -> double2 {
          return (a < ri && k < de) ? A1[h * DM * DS + a * DS + k] : make_double2(0.0, 0.0);
        };
        auto fb = [&](int k, int kp) -> double2 {
          return (k < de && kp < chi) ? A0[h * DM * DS + k * DS + kp] : make_double2(0.0, 0.0);
        };
        cgemm_tile(0, 0, de, fa, fb, cr, ci);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double is = li < chi ? 1.0 / sig[perm[li]] : 0.0;
          Xs[h][lk + 4 * r][li] = cscale(make_double2(cr[r], ci[r]), is);
        }
        wave_lds_sync();
        auto fc = [&](int k, int a) -> double2 {
          return (k < de && a < ri) ? A1[h * DM * DS + a * DS + k] : make_double2(0.0, 0.0);
        };
        auto fd = [&](int a, int kp) -> double2 { return a < ri ? cconj(Xs[h][a][kp]) : make_double2(0.0, 0.0); };
        cgemm_tile(0, 0, ri, fc, fd, cr, ci);
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r) Xs[h][lk + 4 * r][li] = make_double2(cr[r], ci[r]);
      }
      __syncthreads();
      // T_j^(t) = lambda/sigma sum_s g(s,t) Y_s
      for (int idx = tid; idx < 256; idx += NT) {
        const int k = idx >> 4, kp = idx & 15;
        if (k < de && kp < chi) {
          const double2 y0 = Xs[0][k][kp], y1 = Xs[1][k][kp];
          const double f = lam_old[k] / sig[perm[kp]];
          putT(2, k, kp, cscale(cadd(cmul(g00, y0), cmul(g10, y1)), f));
          putT(3, k, kp, cscale(cadd(cmul(g01, y0), cmul(g11, y1)), f));
        }
      }
    }
  }
  if (BWD && !ACC) {
    // the other set of singular vectors for every triplet above kRecTau, through Theta'
    __syncthreads();
    const int ld = 2 * D;
    double2* Ug = st.bU + (int64_t)slot * ld * ld;
    double2* Vg = st.bV + (int64_t)slot * ld * ld;
    const double2* Th = st.wsb + (int64_t)slot * adj_scratch(D) + (int64_t)32 * D * D;  // [2D][2D], formed above
    const double smax = sig[perm[0]];
    const int mO = trans ? n0 : m0;  // rows of the recovered side
    const int kI = trans ? m0 : n0;  // inner dimension
    // O = Theta' V (have V: U = O / sigma) or O = Theta'^H U (have U: V = O / sigma) on the FP64
    // matrix cores, 16 x 16 output tiles over the waves (lane l holds A[l % 16][l / 16] and
    // B[l / 16][l % 16] and receives D[l / 16 + 4 r][l % 16]); triplets at or below kRecTau are zero
    {
      typedef double d4 __attribute__((ext_vector_type(4)));
      const int l = tid & 63, wv = tid >> 6, li = l & 15, lk = l >> 4;
      const int tn = (nB + 15) >> 4, ntile = ((mO + 15) >> 4) * tn, ks = (kI + 3) >> 2;
      const double2* Jv = trans ? Ug : Vg;  // the Jacobi side, [inner][k]
      for (int tile = wv; tile < ntile; tile += NT / 64) {
        const int ti = tile / tn, tj = tile - (tile / tn) * tn;
        const int i = 16 * ti + li, j = 16 * tj + li;
        d4 cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
        for (int s0 = 0; s0 < ks; s0 += 4) {
          double2 a[4], bb[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int kk = 4 * (s0 + u) + lk;
            a[u] = make_double2(0.0, 0.0);
            bb[u] = make_double2(0.0, 0.0);
            if (i < mO && kk < kI) a[u] = trans ? cconj(Th[kk * ld + i]) : Th[i * ld + kk];
            if (j < nB && kk < kI) bb[u] = Jv[kk * ld + j];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (s0 + u < ks) {
              cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, bb[u].x, cr, 0, 0, 0);
              cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[u].y, bb[u].y, cr, 0, 0, 0);
              ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].x, bb[u].y, ci, 0, 0, 0);
              ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].y, bb[u].x, ci, 0, 0, 0);
            }
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rr = 16 * ti + lk + 4 * r, k = 16 * tj + li;
          if (rr < mO && k < nB) {
            const double sv = sig[perm[k]];
            (trans ? Vg : Ug)[rr * ld + k] =
                sv > kRecTau * smax ? cscale(make_double2(cr[r], ci[r]), 1.0 / sv) : make_double2(0.0, 0.0);
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------ K3: re-absorb

template <typename CT, int DM = kMaxD>
__global__ __launch_bounds__(256) void k_reabsorb(DevState st, const int32_t* __restrict__ items, int first,
                                                  int blocks_per_slice) {
  int slot, sp, rb;  // sp = side * 2 + slice
  row_task(st, blockIdx.x, blocks_per_slice, slot, sp, rb);
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

  __shared__ CT Ts[DM][DM + 1];
  __shared__ CT Gs[kRowBlock][DM + 1];
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

// ------------------------------------------------------------------ K3 (complex64): re-absorb on the matrix cores

// Gamma'^(p) = Gamma^(p) T^(p) for complex64 storage, as four real products per complex one on
// v_mfma_f32_16x16x4f32.  With that instruction, lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16] and receives D[4 (l / 16) + r][l % 16], r = 0..3.  The lane that holds
// Gamma[m][k] in one orientation (A = Gamma, B = T) holds the same element in the other
// (A = T^T, B = Gamma^T), and likewise for T, so the operand registers do not depend on the
// orientation; it is chosen per site layout so that the 16 lanes sharing an output register
// store 16 consecutive addresses: C = Gamma T when the bond leg is the contiguous one,
// C^T = T^T Gamma^T when the rows are.  Each wave owns TPW tiles of 16 rows and every bond
// column (at most 32); operands go from global memory straight to registers.  STREAM marks the
// site-tensor rows nontemporal (read and written once, past the caches) for states far larger
// than the L2 caches.
template <int TPW, int DMX = kMaxD, bool STREAM = false>
__global__ __launch_bounds__(256) void k_reabsorb_mfma(DevState st, const int32_t* __restrict__ items, int first,
                                                       int blocks_per_slice) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int RB = 64 * TPW;  // rows per workgroup
  constexpr int KK = DMX / 4;   // k steps of 4 at the largest bond
  constexpr int NT = DMX / 16;  // column tiles of 16 at the largest bond
  int slot, sp, rb;  // sp = side * 2 + slice
  row_task(st, blockIdx.x, blocks_per_slice, slot, sp, rb);
  const int side = sp >> 1, p = sp & 1;
  const int e = items[first + slot];
  const EdgeInfo& E = st.edges[e];
  const SideInfo& S = E.side[side];
  const int D = st.D;
  const int d1 = S.oth[0] >= 0 ? st.chi[S.oth[0]] : 1;
  const int d2 = S.oth[1] >= 0 ? st.chi[S.oth[1]] : 1;
  const int M = d1 * d2;
  if (rb * RB >= M) return;
  const SlotMeta meta = st.meta[slot];
  const int de = meta.de_old;
  const int ncol = max(de, meta.chi_new);  // columns that may be non-zero before or after
  const int ks = (de + 3) >> 2;              // k steps of 4
  const int nt = (ncol + 15) >> 4;           // column tiles of 16
  float2* gam = reinterpret_cast<float2*>(st.gamma);
  const float2* T = reinterpret_cast<const float2*>(st.tbuf) + rbuf_off(st, slot, side, p);
  const int64_t base = S.goff + p * S.pstride;
  const int rstride = d2 > 1 ? S.so[1] : S.so[0];
  const bool bond_major = S.sq == 1 || rstride != 1;  // C = Gamma T (else C^T = T^T Gamma^T)
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = l & 15, lk = l >> 4;

  // T[4 kk + lk][16 t + li]: the same registers serve as B (first form) or A (second form)
  float tr[KK][NT], ti[KK][NT];
#pragma unroll
  for (int kk = 0; kk < KK; ++kk)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int k = 4 * kk + lk, c = 16 * t + li;
      float2 v = make_float2(0.f, 0.f);
      if (k < de && c < ncol) v = T[k * D + c];
      tr[kk][t] = v.x;
      ti[kk][t] = v.y;
    }
  auto row_off = [&](int m) -> int64_t {
    const int o1 = m / d2, o2 = m - (m / d2) * d2;
    return base + (int64_t)o1 * S.so[0] + (int64_t)o2 * S.so[1];
  };
  // every tile's rows are loaded before the first product (memory-level parallelism); a tile
  // past the last row loads nothing and is skipped below
  float gr[TPW][KK], gi[TPW][KK];
#pragma unroll
  for (int tile = 0; tile < TPW; ++tile) {
    const int row0 = rb * RB + (wave * TPW + tile) * 16;
    const int m = row0 + li;
    const int64_t ro = m < M ? row_off(m) : 0;
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
      const int k = 4 * kk + lk;
      float2 v = make_float2(0.f, 0.f);
      if (m < M && k < de) v = ld_c64(&gam[ro + (int64_t)k * S.sq], STREAM);
      gr[tile][kk] = v.x;
      gi[tile][kk] = v.y;
    }
  }
#pragma unroll
  for (int tile = 0; tile < TPW; ++tile) {
    const int row0 = rb * RB + (wave * TPW + tile) * 16;
    if (row0 >= M) break;
    // three real products per complex one: P1 = Gr Tr, P2 = Gi Ti, P3 = (Gr + Gi)(Tr + Ti);
    // Re C = P1 - P2, Im C = P3 - P1 - P2
    f4 q1[NT], q2[NT], q3[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      q1[t] = (f4){0.f, 0.f, 0.f, 0.f};
      q2[t] = (f4){0.f, 0.f, 0.f, 0.f};
      q3[t] = (f4){0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
      if (kk < ks) {
        const float gs = gr[tile][kk] + gi[tile][kk];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          if (t < nt) {
            const float ts = tr[kk][t] + ti[kk][t];
            if (bond_major) {  // C[m][k'] = sum_k Gamma[m][k] T[k][k']
              q1[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(gr[tile][kk], tr[kk][t], q1[t], 0, 0, 0);
              q2[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(gi[tile][kk], ti[kk][t], q2[t], 0, 0, 0);
              q3[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(gs, ts, q3[t], 0, 0, 0);
            } else {           // C^T[k'][m] = sum_k T^T[k'][k] Gamma^T[k][m]
              q1[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(tr[kk][t], gr[tile][kk], q1[t], 0, 0, 0);
              q2[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ti[kk][t], gi[tile][kk], q2[t], 0, 0, 0);
              q3[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ts, gs, q3[t], 0, 0, 0);
            }
          }
        }
      }
    }
    f4 cr[NT], ci[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      cr[t] = q1[t] - q2[t];
      ci[t] = q3[t] - q1[t] - q2[t];
    }
    // the rows of this tile were read into registers above; write the new rows.  A lane's rows
    // are m0, m0 + 1, ... (first form) or the single row m0 (second form): one division, then
    // the other-leg indices (o1, o2) step forward.
    const int m0 = bond_major ? row0 + 4 * lk : row0 + li;
    int o1 = m0 / d2, o2 = m0 - (m0 / d2) * d2;
    int64_t roff[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      roff[r] = base + (int64_t)o1 * S.so[0] + (int64_t)o2 * S.so[1];
      if (bond_major && ++o2 == d2) {
        o2 = 0;
        ++o1;
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (t < nt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = bond_major ? m0 + r : m0;
          const int kp = bond_major ? 16 * t + li : 16 * t + 4 * lk + r;
          if (m < M && kp < ncol)
            st_c64(&gam[roff[bond_major ? r : 0] + (int64_t)kp * S.sq], make_float2(cr[t][r], ci[t][r]), STREAM);
        }
      }
    }
  }
}

// ------------------------------------------------------------------ RX layer

// Gamma_v[0] <- c Gamma_v[0] - i s Gamma_v[1];  Gamma_v[1] <- -i s Gamma_v[0] + c Gamma_v[1]
template <typename CT>
__global__ __launch_bounds__(256) void k_rx(DevState st, int chunk_first, int advance) {
  // the RX layer that opens a recorded step advances the step counter (the readout that closes
  // the step writes history row counter - 1)
  if (advance && blockIdx.x == 0 && threadIdx.x == 0) *st.step_ctr += 1;
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

template <typename CT, int DM = kMaxD>
__global__ __launch_bounds__(256) void k_expect_z(DevState st, int v_first, int record) {
  const int v = v_first + blockIdx.x;
  const VertexInfo& V = st.verts[v];
  const int D = st.D;
  __shared__ double lw[kMaxDeg][DM];
  __shared__ double red0[4], red1[4];
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
  // threads take the inner legs j (their weight computed once, loads coalesced across threads)
  // and loop over the outermost leg a; with fewer inner indices than threads (one or two legs)
  // the threads form G groups of `inner`, group g taking a = g, g + G, ...
  int64_t inner = 1;
  for (int l = 1; l < V.deg; ++l) inner *= D;
  const int na = V.deg >= 1 ? D : 1;
  const int64_t ps = inner * na;
  const CT* gam = reinterpret_cast<const CT*>(st.gamma) + V.goff;
  auto weight = [&](int64_t j) {
    double w = 1.0;
    int64_t rest = j;
    for (int l = V.deg - 1; l >= 1; --l) {
      const int k = (int)(rest % D);
      rest /= D;
      w *= lw[l][k];
    }
    return w;
  };
  double r0 = 0.0, r1 = 0.0;
  if (inner >= (int64_t)blockDim.x) {
    for (int64_t j = tid; j < inner; j += blockDim.x) {
      const double w = weight(j);
      for (int a = 0; a < na; ++a) {
        const double wa = V.deg >= 1 ? w * lw[0][a] : w;
        const int64_t i = (int64_t)a * inner + j;
        r0 += cabs2(to_d2(gam[i])) * wa;
        r1 += cabs2(to_d2(gam[i + ps])) * wa;
      }
    }
  } else {
    const int G = (int)(blockDim.x / inner), g = tid / (int)inner;
    if (g < G) {
      const int64_t j = tid - (int64_t)g * inner;
      const double w = weight(j);
      for (int a = g; a < na; a += G) {
        const double wa = V.deg >= 1 ? w * lw[0][a] : w;
        const int64_t i = (int64_t)a * inner + j;
        r0 += cabs2(to_d2(gam[i])) * wa;
        r1 += cabs2(to_d2(gam[i + ps])) * wa;
      }
    }
  }
  r0 = group_sum_dpp(r0, 64);
  r1 = group_sum_dpp(r1, 64);
  if ((tid & 63) == 0) {
    red0[tid >> 6] = r0;
    red1[tid >> 6] = r1;
  }
  __syncthreads();
  if (tid == 0) {
    const double a = red0[0] + red0[1] + red0[2] + red0[3], b = red1[0] + red1[1] + red1[2] + red1[3];
    const double zv = (a - b) / (a + b);
    if (!isfinite(zv)) flag_status(st.status, kStatusNonFinite);
    st.z[v] = zv;
    if (record) {
      const int row = *st.step_ctr - 1;  // the step's RX layer has advanced the counter
      if (row >= 0 && row < st.max_steps) st.hist[(int64_t)row * st.NV + v] = zv;
    }
  }
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
  if (gid < 4) st.stats[gid] = 0;
}

// ------------------------------------------------------------------ host-side launchers

// complex64 re-absorb: TPW tiles of 16 rows per wave as tuned (8, 4, 2 or 1)
template <int DMX, bool STREAM>
static void launch_reabsorb_mfma(const DevState& st, const int32_t* items, int first, int count, hipStream_t stream) {
  const int tpw = st.tune_rb == 8 ? 8 : st.tune_rb == 4 ? 4 : st.tune_rb == 2 ? 2 : 1;
  const int bps = (st.D * st.D + 64 * tpw - 1) / (64 * tpw);
  const dim3 grid(row_grid(st, count, bps));
  if (tpw == 8)
    hipLaunchKernelGGL((k_reabsorb_mfma<8, DMX, STREAM>), grid, dim3(256), 0, stream, st, items, first, bps);
  else if (tpw == 4)
    hipLaunchKernelGGL((k_reabsorb_mfma<4, DMX, STREAM>), grid, dim3(256), 0, stream, st, items, first, bps);
  else if (tpw == 2)
    hipLaunchKernelGGL((k_reabsorb_mfma<2, DMX, STREAM>), grid, dim3(256), 0, stream, st, items, first, bps);
  else
    hipLaunchKernelGGL((k_reabsorb_mfma<1, DMX, STREAM>), grid, dim3(256), 0, stream, st, items, first, bps);
}

template <typename CT>
static hipError_t launch_set(int which, const DevState& st, const int32_t* items, int first, int count,
                             int blocks_per_slice, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  constexpr bool kAccumulate = sizeof(CT) == sizeof(double2);  // complex128 path keeps the rotations
  if (st.D > kMaxD) {
    // bond dimensions 33..64: R factors as below at 64 columns, the two-site SVD in k_svd_big
    switch (which) {
      case 1:
        if constexpr (sizeof(CT) == sizeof(float2))
          hipLaunchKernelGGL(k_absorb_gram<kMaxDBig>, dim3(count * 4), dim3(256), 0, stream, st, items, first);
        else
          hipLaunchKernelGGL((k_absorb_qr<CT, kMaxDBig, 32>), dim3(count * 4), dim3(256), 0, stream, st, items, first);
        break;
      case 2:
        return launch_svd_big(sizeof(CT) == sizeof(double2), st, items, first, count, stream);
      case 3:
        if constexpr (sizeof(CT) == sizeof(float2)) {
          if (st.stream_gamma)
            launch_reabsorb_mfma<kMaxDBig, true>(st, items, first, count, stream);
          else
            launch_reabsorb_mfma<kMaxDBig, false>(st, items, first, count, stream);
        } else {
          hipLaunchKernelGGL((k_reabsorb<CT, kMaxDBig>), dim3(row_grid(st, count, blocks_per_slice)), dim3(256), 0, stream, st,
                             items, first, blocks_per_slice);
        }
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (which) {
    case 1:
      if constexpr (sizeof(CT) == sizeof(float2)) {
        if (st.D <= 16)
          hipLaunchKernelGGL(k_absorb_gram<16>, dim3(count * 4), dim3(256), 0, stream, st, items, first);
        else
          hipLaunchKernelGGL(k_absorb_gram<32>, dim3(count * 4), dim3(256), 0, stream, st, items, first);
        break;
      }
      if (st.D <= 16) {
        if (st.tune_qr == 8)
          hipLaunchKernelGGL((k_absorb_qr<CT, 16, 8>), dim3(count * 4), dim3(256), 0, stream, st, items, first);
        else
          hipLaunchKernelGGL((k_absorb_qr<CT, 16, 16>), dim3(count * 4), dim3(256), 0, stream, st, items, first);
      } else {
        if (st.tune_qr == 8)
          hipLaunchKernelGGL((k_absorb_qr<CT, 32, 8>), dim3(count * 4), dim3(256), 0, stream, st, items, first);
        else
          hipLaunchKernelGGL((k_absorb_qr<CT, 32, 16>), dim3(count * 4), dim3(256), 0, stream, st, items, first);
      }
      break;
    case 2:
      if (st.D <= 16 && st.tune_svd == 64)
        hipLaunchKernelGGL((k_theta_svd<CT, 64, 32, kAccumulate>), dim3(count), dim3(64), 0, stream, st, items,
                           first);
      else if (st.D <= 16)
        hipLaunchKernelGGL((k_theta_svd<CT, 256, 32, kAccumulate>), dim3(count), dim3(256), 0, stream, st, items,
                           first);
      else
        hipLaunchKernelGGL((k_theta_svd<CT, 256, 64, kAccumulate>), dim3(count), dim3(256), 0, stream, st, items,
                           first);
      break;
    case 3:
      if constexpr (sizeof(CT) == sizeof(float2)) {
        if (st.stream_gamma)
          launch_reabsorb_mfma<kMaxD, true>(st, items, first, count, stream);
        else
          launch_reabsorb_mfma<kMaxD, false>(st, items, first, count, stream);
      } else {
        hipLaunchKernelGGL(k_reabsorb<CT>, dim3(row_grid(st, count, blocks_per_slice)), dim3(256), 0, stream, st, items,
                           first, blocks_per_slice);
      }
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

// The forward SVD update that also keeps every singular triplet and float64 T (reverse sweep).
hipError_t launch_svd_bwd(bool c128, const DevState& st, const int32_t* items, int first, int count,
                          hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (c128) {
    if (st.D <= 16 && st.tune_svd == 64)
      hipLaunchKernelGGL((k_theta_svd<double2, 64, 32, true, true>), dim3(count), dim3(64), 0, stream, st, items,
                         first);
    else if (st.D <= 16)
      hipLaunchKernelGGL((k_theta_svd<double2, 256, 32, true, true>), dim3(count), dim3(256), 0, stream, st, items,
                         first);
    else
      hipLaunchKernelGGL((k_theta_svd<double2, 256, 64, true, true>), dim3(count), dim3(256), 0, stream, st, items,
                         first);
  } else {
    if (st.D <= 16 && st.tune_svd == 64)
      hipLaunchKernelGGL((k_theta_svd<float2, 64, 32, false, true>), dim3(count), dim3(64), 0, stream, st, items,
                         first);
    else if (st.D <= 16)
      hipLaunchKernelGGL((k_theta_svd<float2, 256, 32, false, true>), dim3(count), dim3(256), 0, stream, st, items,
                         first);
    else
      hipLaunchKernelGGL((k_theta_svd<float2, 256, 64, false, true>), dim3(count), dim3(256), 0, stream, st, items,
                         first);
  }
  return hipGetLastError();
}

hipError_t launch_rx(bool c128, const DevState& st, int chunk_first, int n_chunks, int advance, hipStream_t stream) {
  if (n_chunks <= 0) return hipSuccess;
  if (c128) hipLaunchKernelGGL(k_rx<double2>, dim3(n_chunks), dim3(256), 0, stream, st, chunk_first, advance);
  else hipLaunchKernelGGL(k_rx<float2>, dim3(n_chunks), dim3(256), 0, stream, st, chunk_first, advance);
  return hipGetLastError();
}

hipError_t launch_expect_z(bool c128, const DevState& st, int v_first, int n_verts, int record, hipStream_t stream) {
  if (n_verts <= 0) return hipSuccess;
  if (st.D > kMaxD) {
    if (c128) hipLaunchKernelGGL((k_expect_z<double2, kMaxDBig>), dim3(n_verts), dim3(256), 0, stream, st, v_first, record);
    else hipLaunchKernelGGL((k_expect_z<float2, kMaxDBig>), dim3(n_verts), dim3(256), 0, stream, st, v_first, record);
    return hipGetLastError();
  }
  if (c128) hipLaunchKernelGGL(k_expect_z<double2>, dim3(n_verts), dim3(256), 0, stream, st, v_first, record);
  else hipLaunchKernelGGL(k_expect_z<float2>, dim3(n_verts), dim3(256), 0, stream, st, v_first, record);
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
