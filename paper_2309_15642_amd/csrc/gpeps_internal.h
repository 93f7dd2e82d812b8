// Internal layout shared by the host driver and the HIP kernels of libgpeps.
//
// Site tensors (all instances, all qubits) live in one array of complex
// numbers (float2 for GPEPS_C64_F64SVD, double2 for GPEPS_C128).  Qubit v of
// degree k owns 2 * D^k consecutive elements laid out [s][l_0]...[l_{k-1}]:
// the physical index s is outermost (stride D^k) and the virtual legs follow
// in ascending incident-edge id, leg l having stride D^(k-1-l).  Every leg is
// padded to D = d_max; only the leading chi_e entries of leg e are active and
// every entry outside the active box is exactly zero.  Bond weights lambda_e
// are float64 [D] per edge (zeros past chi_e).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpeps {

constexpr int kMaxDeg = 3;
constexpr int kMaxD = 32;      // largest d_max of the LDS-resident kernels (adjoint and BP included)
constexpr int kMaxDBig = 64;   // largest d_max: 32 < d_max <= 64 runs the forward on k_svd_big
// Complex64 path: singular triplets below this fraction of the largest are at the level where
// the vector recovered as Theta' v / sigma is rounding noise; the reverse sweep neither recovers
// nor retains them.
constexpr double kRecTau = 1e-9;
constexpr int kRowBlock = 64;  // rows of a site matrix per re-absorb workgroup
// Size of the device-resident array that holds the BP messages and residual word of
// gpeps_bp_expect_z_noalloc (64 MiB: 2 x 2 NE D^2 complex float64 + 256 B must fit).
constexpr size_t kBpScratchBytes = size_t(64) << 20;
constexpr int kQrChunk = 128;  // rows of a site matrix per Householder chunk

// Status-word bits set by the kernels (checked by the host at sync points).
constexpr int kStatusNonFinite = 1;
constexpr int kStatusNoConverge = 2;
constexpr int kStatusZeroTheta = 4;

// One end of an edge, seen from that edge.
struct SideInfo {
  int64_t goff;     // element offset of the qubit's tensor
  int64_t pstride;  // element stride of the physical index (D^deg)
  int32_t deg;      // degree of the qubit
  int32_t sq;       // element stride of this edge's leg
  int32_t oth[2];   // global ids of the qubit's other edges, -1 if absent
  int32_t so[2];    // element strides of those legs (0 if absent)
};

struct EdgeInfo {
  SideInfo side[2];  // side 0 = lower vertex id, side 1 = higher
  int32_t inst;
  int32_t pad;
};

struct VertexInfo {
  int64_t goff;
  int32_t deg;
  int32_t inst;
  int32_t leg[kMaxDeg];  // global edge ids in leg order, -1 if absent
  int32_t pad;
};

struct InstParam {
  double rx_c, rx_s;  // cos(theta_h / 2), sin(theta_h / 2)
  double g_c, g_s;    // cos(theta_J / 2), sin(theta_J / 2): g(s,t) = g_c - i g_s z_s z_t
};

// Per work-item bookkeeping written by the SVD kernel for the re-absorb kernel.
// Complex float64 entries of per-item adjoint scratch for bond dimension cap D.
__host__ __device__ inline int64_t adj_scratch(int D) { return (int64_t)48 * D * D; }

// Per-item HBM scratch of k_svd_big (d_max > 32), in double2 entries: Theta' [128][128], the
// pivoted R factor [128][128], and [128][64] for the column exchange and then the recovered
// singular-vector set.
__host__ __device__ inline int64_t big_scratch(int /*D*/) {
  return (int64_t)2 * (2 * kMaxDBig) * (2 * kMaxDBig) + (int64_t)2 * kMaxDBig * kMaxDBig;
}

struct SlotMeta {
  int32_t de_old;   // bond dimension of the edge before the update
  int32_t chi_new;  // bond dimension after truncation
  int32_t pad[2];
};

// Everything a kernel needs, passed by value.
struct DevState {
  void* gamma;
  double* lam;            // [NE][D]
  int32_t* chi;           // [NE]
  const EdgeInfo* edges;  // [NE]
  const VertexInfo* verts;  // [NV]
  const InstParam* inst;  // [n_inst]
  double2* rbuf;          // [slots][2 sides][2 slices][D][D] float64 R factors
  void* tbuf;             // [slots][2][2][D][D] re-absorb matrices (storage precision)
  int64_t* stats;         // [4] Jacobi sweeps total, SVD count, max sweeps, non-converged count
  // adjoint (reverse sweep) only
  double2* bU;            // [slots][2D][2D] all left singular vectors of Theta' (row stride 2D)
  double2* bV;            // [slots][2D][2D] all right singular vectors
  double* bS;             // [slots][2D] singular values, descending
  double2* t64;           // [slots][2][2][D][D] float64 re-absorb matrices
  double2* gbar;          // adjoint of the site tensors, float64 complex, same layout as gamma
  double* lbar;           // [NE][D] adjoint of lambda
  double* thbar;          // [n_inst][2] dL/dtheta_h, dL/dtheta_J
  double* gpart;          // [NE + RX chunks] per-edge theta_J and per-chunk theta_h accumulators
  double* wbar;           // [slots][2 sides][2 slices][D^2] per-row w-bar of the edge adjoint
  double2* wsb;           // [slots][adj_scratch(D)] small-matrix scratch of the edge adjoint
  double2* big;           // [slots][big_scratch(D)] scratch of k_svd_big (d_max > 32 only)
  int32_t* ymode;         // [slots][4] QR-adjoint mode per (end, slice): 0 A-bar = A Y, 1 A-bar = Y
  const double* dldz;     // [NV] dL/d<Z_v>
  SlotMeta* meta;         // [slots]
  double* z;              // [NV]
  double* hist;           // [max_steps][NV]
  double2* bp_msg;        // [2][2 NE][D][D] BP messages, two buffers; slot 2e+d: from end d into end 1-d
  unsigned long long* bp_res;  // [1] largest change of a BP message in the last iteration (double bits)
  int32_t* step_ctr;      // device step counter (history row)
  int32_t* status;        // device status word
  const int64_t* chunks;  // RX chunk table: (vertex << 32) | chunk
  const int32_t* inst_vb; // [n_inst + 1] first qubit of every instance (and the total)
  double* mean;           // [n_inst] magnetisation: mean <Z> of every instance
  // launches over one whole colour class: the (item, end) pairs of the class as slot * 2 + end,
  // stored with those whose site has at most one other leg (one block of rows per slice) first,
  // then those with two other legs (the decodes dispatch the latter first); nullptr for a launch
  // over part of a class
  const int32_t* rlist;
  int32_t rl_light, rl_heavy;
  const double* dldm;     // [n_inst] dL/d(magnetisation) of the mean-<Z> loss (adjoint only)
  int32_t n_inst;
  int32_t D;
  int32_t NV;
  int32_t NE;
  int32_t max_sweeps;
  int32_t max_steps;
  int32_t tune_rb;        // complex64 re-absorb: 16-row tiles per wave (1, 2 or 4); autotuned
  int32_t tune_qr;        // QR reduction: rows per lane per chunk (8 or 16); autotuned
  int32_t tune_svd;       // SVD workgroup size for bonds up to 16 (64 or 256); autotuned
  int32_t stream_gamma;   // 1: the site tensors far exceed the L2 caches, so the re-absorb streams
                          //    its rows past them (nontemporal loads and stores)
  double trunc_rel;
};

}  // namespace gpeps
