// Two-site update for bond dimensions 33..64 (Results A and "Long time evolution": chi up to
// several hundred in the paper), gfx950.
//
// At D <= 32 the whole two-site matrix Theta' [2 r_i x 2 r_j] (<= 64 x 64 float64 complex, 64 KB)
// is held in LDS by k_theta_svd.  At D = 64 it is 128 x 128 (256 KB), more than the 160 KB of LDS
// of a CU, so this kernel keeps it where it fits:
//   * Theta' is formed once into a per-item HBM scratch (row-major, leading dimension 128) and
//     stays there for the recovery of the second vector set;
//   * the matrix B whose columns are orthogonalised (B = Theta' or Theta'^H, whichever has fewer
//     columns) lives in registers: 512 threads, 8 lanes per column pair, 16 rows per lane, the
//     stationary and the moving column of every pair (128 VGPRs of data per lane);
//   * one-sided (Hestenes) Jacobi with the pairing {c, c ^ m} of the D <= 32 complex64 kernel:
//     blocks of rounds of equal highest bit hb of m, low bits in Gray-code order, so between
//     rounds every moving column passes to the lane group g ^ 2^b (b the changed bit): a lane
//     permutation inside a wave (lane ^ 8, 16, 32), an LDS exchange (64 columns, 128 KB) across
//     waves; between blocks every column goes to its new owner through LDS (column ids < 64) and
//     the item's HBM scratch (ids >= 64);
//   * B is first reduced by Householder QR with column pivoting, B P = Q R (columns in registers,
//     4 lanes each; the pivot column goes through LDS every step), and the Jacobi iteration runs
//     on X = R^H (nB x nB), whose orthogonalised columns are B's right singular vectors with rows
//     permuted by P: the preconditioning of the D <= 32 complex64 kernel, which gives those
//     vectors to high relative accuracy and cuts the sweeps;
//   * after convergence the kept columns, normalised, give one singular-vector set (staged in
//     LDS); the other set is recovered from the stored Theta' as Theta' v / sigma (or
//     Theta'^H u / sigma), accurate to ~2^-52 sigma_0 / sigma for every kept value, and the four
//     re-absorb matrices T follow as in k_theta_svd:
//       T_i^(s)[k,k'] = lambda_k / sigma_k' sum_{t,b} g(s,t) R_j^(t)[b,k] V[(t,b),k'],
//       T_j^(t)[k,k'] = lambda_k / sigma_k' sum_{s,a} g(s,t) conj(U[(s,a),k']) R_i^(s)[a,k].
// A sweep ends the iteration when it rotates nothing, or (complex64 storage) when all its
// rotations had |g|^2 <= 1e-8 al be, as in k_theta_svd.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "gpeps_device.h"
#include "gpeps_internal.h"

namespace gpeps {

namespace {

constexpr int kBT = 512;                 // threads per item
constexpr int kBN = 2 * kMaxDBig;        // 128: largest side of Theta'
constexpr int kBLJ = 8;                  // lanes per column pair
constexpr int kBRPL = kBN / kBLJ;        // 16 rows per lane
constexpr int kBGroups = kBT / kBLJ;     // 64 lane groups (column pairs)
constexpr double kQuietBigC64 = 1e-8;    // (1e-4)^2, as the complex64 path of k_theta_svd

__device__ __forceinline__ int ins_bit(int g, int hb, int bit) {
  return ((g >> hb) << (hb + 1)) | (bit << hb) | (g & ((1 << hb) - 1));
}

// The 16 rows of the moving column held by this lane, exchanged with lane ^ OFF.
template <int OFF>
__device__ __forceinline__ void move_col(double2 (&x)[kBRPL], double& n2) {
#pragma unroll
  for (int u = 0; u < kBRPL; ++u) {
    const unsigned long long bx = (unsigned long long)__double_as_longlong(x[u].x);
    const unsigned long long by = (unsigned long long)__double_as_longlong(x[u].y);
    unsigned w0 = (unsigned)(bx & 0xffffffffull), w1 = (unsigned)(bx >> 32);
    unsigned w2 = (unsigned)(by & 0xffffffffull), w3 = (unsigned)(by >> 32);
    lane_xor2<OFF>(w0, w1);
    lane_xor2<OFF>(w2, w3);
    x[u] = make_double2(__longlong_as_double((long long)(((unsigned long long)w1 << 32) | w0)),
                        __longlong_as_double((long long)(((unsigned long long)w3 << 32) | w2)));
  }
  n2 = lane_xor<OFF>(n2);
}

}  // namespace

template <typename CT>
__global__ __launch_bounds__(kBT) void k_svd_big(DevState st, const int32_t* __restrict__ items, int first) {
  constexpr bool C64 = sizeof(CT) == sizeof(float2);
  __shared__ double2 X[kBGroups][kBN + 1];  // 129 KB: column exchange, then the kept vectors [k'][row]
  __shared__ double nrmx[kBN];          // tracked squared norms by column id (exchanges)
  __shared__ double sig[kBN];
  __shared__ int perm[kBN];
  __shared__ int colid_sh[kBN];  // original column of each pivot position
  __shared__ double lam_old[kMaxDBig];
  __shared__ double red_w[kBT / 64];
  __shared__ int sh_flag[3][2];
  __shared__ int sh_chi;
  __shared__ double sh_norm, sh_floor;

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
  const double2* Rg = st.rbuf + rbuf_off(st, slot, 0, 0);  // blocks i0, i1, j0, j1, each [D][D]
  double2* Tg = st.big + (int64_t)slot * big_scratch(D);  // Theta' [m0][n0], leading dimension kBN
  double2* Rs = Tg + kBN * kBN;                            // R by pivot position: Rs[pos][row]
  double2* Og = Rs + kBN * kBN;                            // exchange, then the other vector set

  if (tid < kMaxDBig) lam_old[tid] = tid < de ? lam_e[tid] : 0.0;
  if (tid < 6) sh_flag[tid >> 1][tid & 1] = 0;

  __syncthreads();  // lam_old
  // Theta'[(s,a)][(t,b)] = g(s,t) sum_k R_i^(s)[a,k] lambda_k R_j^(t)[b,k]: 16 x 16 tiles on the
  // FP64 matrix cores, the waves taking the tiles in turn, operands from the R factors
  {
    double fro = 0.0;
    const int wv = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
    const int tm = (m0 + 15) >> 4, tn = (n0 + 15) >> 4;
    auto fa = [&](int i, int k) -> double2 {
      if (i >= m0 || k >= de) return make_double2(0.0, 0.0);
      const int s = i / ri, a = i - (i / ri) * ri;
      return cscale(Rg[(int64_t)s * D * D + a * D + k], lam_old[k]);
    };
    auto fb = [&](int k, int j) -> double2 {
      if (j >= n0 || k >= de) return make_double2(0.0, 0.0);
      const int t = j / rj, b = j - (j / rj) * rj;
      return Rg[(int64_t)(2 + t) * D * D + b * D + k];
    };
    for (int tile = wv; tile < tm * tn; tile += kBT / 64) {
      const int ti = tile / tn, tj = tile - (tile / tn) * tn;
      cgemm_d4 cr, ci;
      cgemm_tile(16 * ti, 16 * tj, de, fa, fb, cr, ci);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * ti + lk + 4 * r, col = 16 * tj + li;
        if (row < m0 && col < n0) {
          const double2 v = cmul(make_double2(cr[r], ci[r]), gate_phase(ip, row / ri, col / rj));
          Tg[row * kBN + col] = v;
          fro += cabs2(v);
        }
      }
    }
    fro = group_sum_dpp(fro, 64);
    if ((tid & 63) == 0) red_w[tid >> 6] = fro;
  }
  __syncthreads();
  if (tid == 0) {
    double f = 0.0;
    for (int w = 0; w < kBT / 64; ++w) f += red_w[w];
    sh_floor = f * st.trunc_rel * st.trunc_rel * 2.220446049250313e-16;
  }

  // B[c][r] = Theta'[r][c] (not trans) or conj(Theta'[c][r]) (trans), from the HBM copy
  auto b_at = [&](int c, int rr) -> double2 {
    return trans ? cconj(Tg[c * kBN + rr]) : Tg[rr * kBN + c];
  };
  __syncthreads();  // sh_floor

  // Householder QR with column pivoting, B P = Q R (only R is kept).  Column c sits in the
  // registers of lanes 4c .. 4c + 3 (rows ql + 4u); pivoting is virtual (colid records the
  // order).  Every step: the pivot comes from the per-wave candidates of the previous step, its
  // column's rows j.. go through LDS, every group builds the reflector from that copy
  // (bit-identical in all groups) and applies it to its own column, then publishes the next
  // candidate.  The key of a candidate is the squared norm with its 7 lowest mantissa bits
  // replaced by 127 - column (ties within 2^-45 relative go to the lowest column); a zero
  // norm keeps key 0, a column that cannot be chosen has key -1.
  {
    constexpr int LQ = kBT / kBN;  // 4 lanes per column
    constexpr int RQ = kBN / LQ;   // 32 rows per lane
    __shared__ double2 pcol[kBN];
    __shared__ double cand[2][kBT / 64];
    __shared__ int posof[kBN];
    const int qc = tid / LQ, ql = tid - (tid / LQ) * LQ, wv = tid >> 6;
    double2 x[RQ];
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      const int rr = ql + LQ * u;
      x[u] = (qc < nB && rr < mB) ? b_at(qc, rr) : make_double2(0.0, 0.0);
    }
    auto publish = [&](double s2, bool valid, int buf) {
      double key = -1.0;
      if (valid)
        key = s2 > 0.0 ? __longlong_as_double((__double_as_longlong(s2) & ~127ll) | (long long)(127 - qc)) : 0.0;
      const double m = wave_max_uniform(key);
      if ((tid & 63) == 0) cand[buf][wv] = m;
    };
    {
      double s2 = 0.0;
#pragma unroll
      for (int u = 0; u < RQ; ++u) s2 += cabs2(x[u]);
      publish(group_sum_dpp(s2, LQ), qc < nB, 0);
    }
    if (tid < kBN) posof[tid] = -1;
    bool used = false;
    int jP = 0;
    double2 betaP = make_double2(0.0, 0.0);
    __syncthreads();
    int j = 0;
    for (; j < nB; ++j) {
      double best = cand[j & 1][0];
#pragma unroll
      for (int w = 1; w < kBT / 64; ++w) best = fmax(best, cand[j & 1][w]);
      if (!(best > 0.0)) break;  // the remaining columns are zero below row j
      const int P = 127 - (int)(__double_as_longlong(best) & 127ll);
      if (qc == P) {
#pragma unroll
        for (int u = 0; u < RQ; ++u) {
          const int rr = ql + LQ * u;
          if (rr >= j && rr < mB) pcol[rr] = x[u];
        }
        if (ql == 0) posof[P] = j;
      }
      __syncthreads();
      // reflector I - tau v v^H, v = x - beta e_j, beta = -phase(x_j) ||x||, x = rows j.. of the pivot
      const double2 alpha = pcol[j];
      double sb = 0.0;
#pragma unroll
      for (int u = 0; u < RQ; ++u) {
        const int rr = ql + LQ * u;
        if (rr > j && rr < mB) sb += cabs2(pcol[rr]);
      }
      sb = group_sum_dpp(sb, LQ);
      if (qc == P) {
        used = true;
        jP = j;
        betaP = alpha;
      }
      double s2 = 0.0;
      if (sb > 0.0) {
        const double aa2 = cabs2(alpha);
        const double nu2 = aa2 + sb;
        const double nu = nu2 * rsq_nr(nu2);
        const double2 ph = aa2 > 0.0 ? cscale(alpha, rsq_nr(aa2)) : make_double2(1.0, 0.0);
        const double2 beta = cscale(ph, -nu);
        const double2 v0 = csub(alpha, beta);
        const double tau = 2.0 * rcp_nr(cabs2(v0) + sb);
        if (qc == P) betaP = beta;
        if (!used && qc < nB) {
          double wr = 0.0, wi = 0.0;
#pragma unroll
          for (int u = 0; u < RQ; ++u) {
            const int rr = ql + LQ * u;
            if (rr >= j && rr < mB) {
              const double2 g = cmulc(rr == j ? v0 : pcol[rr], x[u]);
              wr += g.x;
              wi += g.y;
            }
          }
          group_sum2_dpp(wr, wi, LQ);
          const double2 f = make_double2(wr * tau, wi * tau);
#pragma unroll
          for (int u = 0; u < RQ; ++u) {
            const int rr = ql + LQ * u;
            if (rr >= j && rr < mB) {
              x[u] = csub(x[u], cmul(rr == j ? v0 : pcol[rr], f));
              if (rr > j) s2 += cabs2(x[u]);
            }
          }
        }
      } else if (!used && qc < nB) {
#pragma unroll
        for (int u = 0; u < RQ; ++u) {
          const int rr = ql + LQ * u;
          if (rr > j && rr < mB) s2 += cabs2(x[u]);
        }
      }
      publish(group_sum_dpp(s2, LQ), !used && qc < nB, (j + 1) & 1);
      __syncthreads();
    }
    // R's pivot columns: beta on the diagonal, zeros below; never-pivoted (zero below row j)
    // columns follow in ascending order
    if (used && qc < nB) {
#pragma unroll
      for (int u = 0; u < RQ; ++u) {
        const int rr = ql + LQ * u;
        if (rr == jP) x[u] = betaP;
        else if (rr > jP) x[u] = make_double2(0.0, 0.0);
      }
    }
    if (tid == 0)
      for (int c = 0, k = j; c < nB; ++c)
        if (posof[c] < 0) posof[c] = k++;
    __syncthreads();
    if (qc < nB) {
      const int pos = posof[qc];
#pragma unroll
      for (int u = 0; u < RQ; ++u) {
        const int rr = ql + LQ * u;
        if (rr < nB) Rs[pos * kBN + rr] = rr < mB ? x[u] : make_double2(0.0, 0.0);
      }
    }
    if (tid < nB) perm[posof[tid]] = tid;  // perm[pos] = original column (reused below for sorting)
    __syncthreads();
    if (tid < nB) colid_sh[tid] = perm[tid];
    __syncthreads();
  }
  // the Jacobi matrix X = R^H (nB x nB): X[c][r] = conj(R(c, r)) = conj(Rs[r][c])
  auto x_at = [&](int c, int rr) -> double2 { return cconj(Rs[rr * kBN + c]); };
  const int pair_id = tid / kBLJ;
  const int lane = tid - pair_id * kBLJ;
  auto xrow = [&](int u) { return lane + kBLJ * u; };
  int K = 1;
  while ((1 << K) < nB) ++K;
  const bool gact = pair_id < (1 << (K - 1));
  const double tol2 = (2.220446049250313e-16 * (double)nB) * (2.220446049250313e-16 * (double)nB);
  double2 xs[kBRPL], xm[kBRPL];  // stationary and moving column of the group
  double ns = 0.0, nm = 0.0;
  int cs_id = ins_bit(pair_id, 0, 0), cm_id = ins_bit(pair_id, 0, 1);
  auto col_norm = [&](const double2 (&x)[kBRPL]) {
    double s2 = 0.0;
#pragma unroll
    for (int u = 0; u < kBRPL; ++u) s2 += cabs2(x[u]);
    return group_sum_dpp(s2, kBLJ);
  };
  // initial assignment (block hb = 0): group g holds columns 2g and 2g + 1
#pragma unroll
  for (int u = 0; u < kBRPL; ++u) {
    const int rr = xrow(u);
    xs[u] = (gact && cs_id < nB && rr < nB) ? x_at(cs_id, rr) : make_double2(0.0, 0.0);
    xm[u] = (gact && cm_id < nB && rr < nB) ? x_at(cm_id, rr) : make_double2(0.0, 0.0);
  }
  const double floor2 = sh_floor * sh_floor;

  // every column to its owner under block hb (ids < 64 through LDS, ids >= 64 through HBM)
  auto redistribute = [&](int hb) {
    auto put = [&](const double2 (&x)[kBRPL], int c, double n2) {
      if (!gact || c >= nB) return;
      double2* dst = c < kBGroups ? &X[c][0] : Og + (int64_t)(c - kBGroups) * kBN;
#pragma unroll
      for (int u = 0; u < kBRPL; ++u) dst[xrow(u)] = x[u];
      if (lane == 0) nrmx[c] = n2;
    };
    put(xs, cs_id, ns);
    put(xm, cm_id, nm);
    __syncthreads();
    cs_id = ins_bit(pair_id, hb, 0);
    cm_id = ins_bit(pair_id, hb, 1);
    auto get = [&](double2 (&x)[kBRPL], int c, double& n2) {
      const bool ok = gact && c < nB;
      const double2* src = c < kBGroups ? &X[c < kBGroups ? c : 0][0] : Og + (int64_t)(c - kBGroups) * kBN;
#pragma unroll
      for (int u = 0; u < kBRPL; ++u) {
        const double2 t = src[xrow(u)];
        x[u] = ok ? t : make_double2(0.0, 0.0);
      }
      n2 = ok ? nrmx[c] : 0.0;
    };
    get(xs, cs_id, ns);
    get(xm, cm_id, nm);
    __syncthreads();
  };

  bool rot = false, big = false;
  int sweep = 0;
  bool converged = nB < 2;
  for (; sweep < st.max_sweeps && !converged; ++sweep) {
    for (int hb = 0; hb < K; ++hb) {
      if (hb == 0) {
        ns = col_norm(xs);
        nm = col_norm(xm);
      }
      const int nt = 1 << hb;
      for (int t = 0; t < nt; ++t) {
        // rotation of the pair (stationary xs, moving xm); branch-free: a pair that is not
        // rotated takes c = 1, s = 0, which leaves both columns and norms bit for bit
        double2 g = cmulc(xs[0], xm[0]);
#pragma unroll
        for (int u = 1; u < kBRPL; ++u) g = cadd(g, cmulc(xs[u], xm[u]));
        double gr = g.x, gi = g.y;
        group_sum2_dpp(gr, gi, kBLJ);
        const double al = ns, be = nm;
        const double g2 = gr * gr + gi * gi;
        const bool ok = gact & (cm_id < nB) & (g2 > tol2 * al * be) & (g2 > floor2);
        const double d = be - al;
        const double h2 = d * d + 4.0 * g2;
        const double rh = C64 ? rsq_nr1(h2) : rsq_nr(h2);  // 1 / h
        const double xx = 0.5 + 0.5 * fabs(d) * rh;
        const double rc = C64 ? rsq_nr1(xx) : rsq_nr(xx);  // 1 / c
        const double f = (d < 0.0 ? -rh : rh) * rc;
        const double cs = ok ? xx * rc : 1.0;
        const double2 sph = ok ? make_double2(gr * f, gi * f) : make_double2(0.0, 0.0);
        const double tg = ok ? g2 * f * rc : 0.0;
#pragma unroll
        for (int u = 0; u < kBRPL; ++u) {
          const double2 bp = xs[u], bq = xm[u];
          xs[u] = csub(cscale(bp, cs), cmulc(sph, bq));
          xm[u] = cadd(cmul(sph, bp), cscale(bq, cs));
        }
        ns = al - tg;
        nm = be + tg;
        rot = rot || ok;
        big = big || (ok && g2 > kQuietBigC64 * al * be);
        if (t + 1 < nt) {
          // the moving column passes to group pair_id ^ 2^bb
          const int bb = __builtin_ctz(t + 1);
          const int mp = (t + 1) ^ ((t + 1) >> 1);
          if (bb == 0) {
            move_col<kBLJ>(xm, nm);
          } else if (bb == 1) {
            move_col<2 * kBLJ>(xm, nm);
          } else if (bb == 2) {
            move_col<4 * kBLJ>(xm, nm);
          } else {
#pragma unroll
            for (int u = 0; u < kBRPL; ++u) X[pair_id][xrow(u)] = xm[u];
            if (lane == 0) nrmx[pair_id] = nm;
            __syncthreads();
            const int src = pair_id ^ (1 << bb);
#pragma unroll
            for (int u = 0; u < kBRPL; ++u) xm[u] = X[src][xrow(u)];
            nm = nrmx[src];
            __syncthreads();
          }
          cm_id = ins_bit(pair_id ^ mp, hb, 1);
        }
      }
      if (hb + 1 == K) {
        if (rot && lane == 0) sh_flag[sweep % 3][0] = 1;
        if (big && lane == 0) sh_flag[sweep % 3][1] = 1;
        if (tid < 2) sh_flag[(sweep + 1) % 3][tid] = 0;
        rot = false;
        big = false;
      }
      if (hb + 1 < K) redistribute(hb + 1);
    }
    __syncthreads();
    converged = (sh_flag[sweep % 3][0] == 0) || (C64 && sh_flag[sweep % 3][1] == 0);
    if (!converged) redistribute(0);
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

  // singular values (norms of the held columns), stable descending order, truncation
  const double s_s = sqrt(col_norm(xs)), s_m = sqrt(col_norm(xm));
  if (lane == 0 && gact) {
    if (cs_id < nB) sig[cs_id] = s_s;
    if (cm_id < nB) sig[cm_id] = s_m;
  }
  __syncthreads();
  for (int c = tid; c < nB; c += kBT) {
    const double sv = sig[c];
    int rank = 0;
    for (int d2 = 0; d2 < nB; ++d2) {
      const double sd = sig[d2];
      rank += (sd > sv) || (sd == sv && d2 < c);
    }
    perm[rank] = c;
  }
  __syncthreads();
  if (tid == 0) {
    const double smax = sig[perm[0]];
    int keep = 0;
    for (int d2 = 0; d2 < nB; ++d2) keep += sig[d2] > st.trunc_rel * smax;
    int chi = keep < D ? keep : D;
    if (chi < 1) chi = 1;
    double nr = 0.0;
    for (int k = 0; k < chi; ++k) nr += sig[perm[k]] * sig[perm[k]];
    nr = sqrt(nr);
    if (!(smax > 0.0)) flag_status(st.status, kStatusZeroTheta);
    if (!isfinite(nr)) flag_status(st.status, kStatusNonFinite);
    sh_chi = chi;
    sh_norm = nr;
    st.meta[slot].de_old = de;
    st.meta[slot].chi_new = chi;
    st.chi[e] = chi;
  }
  __syncthreads();
  const int chi = sh_chi;
  for (int k = tid; k < D; k += kBT) lam_e[k] = k < chi ? sig[perm[k]] / sh_norm : 0.0;

  // kept columns of X, normalised: B's right singular vectors with rows permuted by the pivoting,
  // X[k'][colid[r]] = x[r] / sigma (rows < nB)
  auto stage = [&](const double2 (&x)[kBRPL], int c, double sv) {
    if (!gact || c >= nB) return;
    int rank = 0;
    for (int d2 = 0; d2 < nB; ++d2) {
      const double sd = sig[d2];
      rank += (sd > sv) || (sd == sv && d2 < c);
    }
    if (rank >= chi) return;
    const double inv = sv > 0.0 ? 1.0 / sv : 0.0;
#pragma unroll
    for (int u = 0; u < kBRPL; ++u) {
      const int rr = xrow(u);
      if (rr < nB) X[rank][colid_sh[rr]] = cscale(x[u], inv);
    }
  };
  stage(xs, cs_id, sig[cs_id < nB ? cs_id : 0]);
  stage(xm, cm_id, sig[cm_id < nB ? cm_id : 0]);
  __syncthreads();

  // B's right singular vectors are V of Theta' (B = Theta') or U of Theta' (B = Theta'^H); the
  // other set from the stored Theta': U = Theta' V / sigma or V = Theta'^H U / sigma, into
  // Og[row][k'] (leading dimension kMaxDBig)
  const int mO = trans ? n0 : m0;
  {
    const int wv = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
    const int tm = (mO + 15) >> 4, tn = (chi + 15) >> 4;
    auto fa = [&](int i, int q) -> double2 {
      if (i >= mO || q >= nB) return make_double2(0.0, 0.0);
      return trans ? cconj(Tg[q * kBN + i]) : Tg[i * kBN + q];
    };
    auto fb = [&](int q, int j) -> double2 {
      if (q >= nB || j >= chi) return make_double2(0.0, 0.0);
      return X[j][q];
    };
    for (int tile = wv; tile < tm * tn; tile += kBT / 64) {
      const int ti = tile / tn, tj = tile - (tile / tn) * tn;
      cgemm_d4 cr, ci;
      cgemm_tile(16 * ti, 16 * tj, nB, fa, fb, cr, ci);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = 16 * ti + lk + 4 * r, kp = 16 * tj + li;
        if (rr < mO && kp < chi) {
          const double sv = sig[perm[kp]];
          Og[rr * kMaxDBig + kp] = sv > 0.0 ? cscale(make_double2(cr[r], ci[r]), 1.0 / sv) : make_double2(0.0, 0.0);
        }
      }
    }
  }
  __syncthreads();
  // U[(s,a)][k'] and V[(t,b)][k'] wherever they are
  auto Uv = [&](int row, int kp) -> double2 { return trans ? X[kp][row] : Og[row * kMaxDBig + kp]; };
  auto Vv = [&](int row, int kp) -> double2 { return trans ? Og[row * kMaxDBig + kp] : X[kp][row]; };

  CT* T = reinterpret_cast<CT*>(st.tbuf);
  for (int idx = tid; idx < 4 * de * (D - chi); idx += kBT) {
    const int w = idx / (de * (D - chi));
    const int rem = idx - w * de * (D - chi);
    const int k = rem / (D - chi), kp = chi + rem - (rem / (D - chi)) * (D - chi);
    T[rbuf_off(st, slot, w >> 1, w & 1) + k * D + kp] = from_d2<CT>(make_double2(0.0, 0.0));
  }
  const double2 g00 = gate_phase(ip, 0, 0), g01 = gate_phase(ip, 0, 1);
  const double2 g10 = gate_phase(ip, 1, 0), g11 = gate_phase(ip, 1, 1);
  const double2* RI0 = Rg;
  const double2* RI1 = Rg + (int64_t)D * D;
  const double2* RJ0 = Rg + (int64_t)2 * D * D;
  const double2* RJ1 = Rg + (int64_t)3 * D * D;
  // x_t[k][k'] = sum_b R_j^(t)[b][k] V[(t,b)][k'], y_s[k][k'] = sum_a R_i^(s)[a][k] conj(U[(s,a)][k']):
  // four products per 16 x 16 tile of (k, k'), on the matrix cores
  {
    const int wv = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
    const int tm = (de + 15) >> 4, tn = (chi + 15) >> 4;
    for (int tile = wv; tile < tm * tn; tile += kBT / 64) {
      const int ti = tile / tn, tj = tile - (tile / tn) * tn;
      cgemm_d4 xr[2], xi[2], yr[2], yi[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double2* RJ = h ? RJ1 : RJ0;
        const double2* RI = h ? RI1 : RI0;
        auto fjx = [&](int k, int b) -> double2 {
          return (k < de && b < rj) ? RJ[b * D + k] : make_double2(0.0, 0.0);
        };
        auto fjv = [&](int b, int kp) -> double2 {
          return (b < rj && kp < chi) ? Vv(h * rj + b, kp) : make_double2(0.0, 0.0);
        };
        auto fix = [&](int k, int a) -> double2 {
          return (k < de && a < ri) ? RI[a * D + k] : make_double2(0.0, 0.0);
        };
        auto fiu = [&](int a, int kp) -> double2 {
          return (a < ri && kp < chi) ? cconj(Uv(h * ri + a, kp)) : make_double2(0.0, 0.0);
        };
        cgemm_tile(16 * ti, 16 * tj, rj, fjx, fjv, xr[h], xi[h]);
        cgemm_tile(16 * ti, 16 * tj, ri, fix, fiu, yr[h], yi[h]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = 16 * ti + lk + 4 * r, kp = 16 * tj + li;
        if (k < de && kp < chi) {
          const double2 x0 = make_double2(xr[0][r], xi[0][r]), x1 = make_double2(xr[1][r], xi[1][r]);
          const double2 y0 = make_double2(yr[0][r], yi[0][r]), y1 = make_double2(yr[1][r], yi[1][r]);
          const double f = lam_old[k] / sig[perm[kp]];
          T[rbuf_off(st, slot, 0, 0) + k * D + kp] = from_d2<CT>(cscale(cadd(cmul(g00, x0), cmul(g01, x1)), f));
          T[rbuf_off(st, slot, 0, 1) + k * D + kp] = from_d2<CT>(cscale(cadd(cmul(g10, x0), cmul(g11, x1)), f));
          T[rbuf_off(st, slot, 1, 0) + k * D + kp] = from_d2<CT>(cscale(cadd(cmul(g00, y0), cmul(g10, y1)), f));
          T[rbuf_off(st, slot, 1, 1) + k * D + kp] = from_d2<CT>(cscale(cadd(cmul(g01, y0), cmul(g11, y1)), f));
        }
      }
    }
  }
}

hipError_t launch_svd_big(bool c128, const DevState& st, const int32_t* items, int first, int count,
                          hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (st.D > kMaxDBig || !st.big) return hipErrorInvalidValue;
  if (c128) hipLaunchKernelGGL(k_svd_big<double2>, dim3(count), dim3(kBT), 0, stream, st, items, first);
  else hipLaunchKernelGGL(k_svd_big<float2>, dim3(count), dim3(kBT), 0, stream, st, items, first);
  return hipGetLastError();
}

}  // namespace gpeps
