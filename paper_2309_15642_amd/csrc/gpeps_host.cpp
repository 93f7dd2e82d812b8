// Host driver of libgpeps: the C ABI declared in include/gpeps.h.
//
// Responsibilities: validate graphs and colourings (or colour them), lay the
// caller's workspace out into site tensors, bond weights, tables and scratch,
// build the per-colour-class work lists, and enqueue the kernels -- batched
// (one launch per kernel per colour class, all instances together, a whole
// Trotter step captured once as a hipGraph and replayed) or plain (one edge of
// one instance per launch, no graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/gpeps.h"
#include "gpeps_internal.h"

namespace gpeps {
hipError_t launch_edge_kernel(int which, bool c128, const DevState& st, const int32_t* items, int first, int count,
                              int blocks_per_slice, hipStream_t stream);
hipError_t launch_rx(bool c128, const DevState& st, int chunk_first, int n_chunks, int advance, hipStream_t stream);
hipError_t launch_expect_z(bool c128, const DevState& st, int v_first, int n_verts, int record, hipStream_t stream);
hipError_t launch_bp(bool c128, const DevState& st, int iters, hipStream_t stream);
hipError_t bp_scratch_address(void** ptr);
hipError_t launch_reset(bool c128, const DevState& st, int64_t n_gamma, hipStream_t stream);
hipError_t launch_adjoint(int which, bool c128, const DevState& st, const int32_t* items, int first, int count,
                          int blocks_per_slice, const void* aux, hipStream_t stream);
hipError_t launch_checkpoint(const DevState& st, const void* src, void* dst, int64_t bytes, int64_t slot_bytes,
                             hipStream_t stream);
hipError_t launch_fill_d(double* p, int64_t n, hipStream_t stream);
hipError_t launch_mean_z(const DevState& st, int row, hipStream_t stream);
hipError_t launch_seed_mean(const DevState& st, hipStream_t stream);
hipError_t launch_svd_bwd(bool c128, const DevState& st, const int32_t* items, int first, int count,
                          hipStream_t stream);
}  // namespace gpeps

using namespace gpeps;

namespace {

thread_local std::string g_thread_error;

constexpr int kKinds = 5;
const char* const kKindNames[kKinds] = {"rx", "absorb_qr", "theta_svd", "reabsorb", "expect_z"};

struct Layout {
  // host tables
  std::vector<EdgeInfo> edges;
  std::vector<VertexInfo> verts;
  std::vector<InstParam> inst;
  std::vector<int32_t> items;              // all colour classes concatenated
  std::vector<int> class_begin, class_end;  // per class, into items
  std::vector<int32_t> rlist;               // per class: (slot * 2 + end), light ends stored first
  std::vector<int> rl_begin, rl_light, rl_heavy;
  std::vector<int64_t> chunks;             // RX chunk table
  std::vector<int> inst_chunk_begin, inst_chunk_end;
  std::vector<int> inst_vert_begin, inst_vert_end;
  std::vector<int> inst_edge_begin;
  // class items grouped by instance for plain mode
  int NV = 0, NE = 0, max_items = 0, n_classes = 0;
  size_t class_slots = 1;  // slots per colour class in the per-class buffers
  int64_t n_gamma = 0;
  // workspace offsets (bytes)
  size_t off_gamma = 0, off_lam = 0, off_chi = 0, off_edges = 0, off_verts = 0, off_inst = 0, off_items = 0,
         off_rbuf = 0, off_tbuf = 0, off_stats = 0, off_meta = 0, off_ckpt = 0, off_snap = 0, off_work = 0,
         off_gbar = 0, off_lbar = 0, off_thbar = 0, off_dldz = 0, off_bU = 0, off_bV = 0, off_bS = 0, off_t64 = 0,
         off_wsb = 0, off_ybuf = 0, off_ymode = 0, state_bytes = 0, state_slot = 0, off_z = 0, off_hist = 0, off_ctr = 0, off_chunks = 0,
         off_bp = 0, off_bpres = 0, off_ivb = 0, off_mean = 0, off_dldm = 0, off_big = 0, off_gpart = 0,
         off_wbar = 0, off_rlist = 0;
  size_t total = 0;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// König / Kempe alternating-path edge colouring (bipartite graphs), edge order.
bool kempe_colour(int n, const std::vector<std::pair<int, int>>& ed, std::vector<int32_t>& col, std::string& err) {
  const int m = (int)ed.size();
  std::vector<int> deg(n, 0);
  for (auto& e : ed) {
    deg[e.first]++;
    deg[e.second]++;
  }
  int k = 0;
  for (int d : deg) k = std::max(k, d);
  col.assign(m, -1);
  std::vector<std::vector<int>> at(n, std::vector<int>(std::max(k, 1), -1));
  auto free_at = [&](int x) {
    for (int c = 0; c < k; ++c)
      if (at[x][c] < 0) return c;
    return -1;
  };
  for (int e = 0; e < m; ++e) {
    const int u = ed[e].first, v = ed[e].second;
    const int a = free_at(u), b = free_at(v);
    if (a < 0 || b < 0) {
      err = "edge colouring: no free colour";
      return false;
    }
    int c;
    if (at[v][a] < 0) {
      c = a;
    } else if (at[u][b] < 0) {
      c = b;
    } else {
      std::vector<int> path;
      int x = v, cur = a;
      while (at[x][cur] >= 0) {
        const int f = at[x][cur];
        path.push_back(f);
        const int y = ed[f].first == x ? ed[f].second : ed[f].first;
        if (y == u) {
          err = "edge colouring: graph is not bipartite, pass an explicit colouring";
          return false;
        }
        x = y;
        cur = (cur == a) ? b : a;
      }
      for (int f : path) {
        at[ed[f].first][col[f]] = -1;
        at[ed[f].second][col[f]] = -1;
      }
      for (int f : path) {
        col[f] = (col[f] == a) ? b : a;
        at[ed[f].first][col[f]] = f;
        at[ed[f].second][col[f]] = f;
      }
      c = a;
    }
    col[e] = c;
    at[u][c] = e;
    at[v][c] = e;
  }
  return true;
}

struct GraphTables {
  int n_nodes = 0, n_edges = 0;
  std::vector<std::pair<int, int>> ed;  // (lo, hi)
  std::vector<int32_t> colour;
  std::vector<std::vector<int>> inc;  // ascending incident edge ids
  int n_colours = 0;
};

gpeps_status check_graph(const gpeps_graph& g, GraphTables& t, std::string& err) {
  if (g.n_nodes < 1 || g.n_edges < 0 || (g.n_edges > 0 && !g.edges)) {
    err = "graph: n_nodes must be >= 1 and edges non-NULL";
    return GPEPS_ERR_ARG;
  }
  t.n_nodes = g.n_nodes;
  t.n_edges = g.n_edges;
  t.ed.resize(g.n_edges);
  std::map<std::pair<int, int>, int> seen;
  for (int e = 0; e < g.n_edges; ++e) {
    int u = g.edges[2 * e], v = g.edges[2 * e + 1];
    if (u < 0 || v < 0 || u >= g.n_nodes || v >= g.n_nodes) {
      err = "graph: edge endpoint out of range";
      return GPEPS_ERR_ARG;
    }
    if (u == v) {
      err = "graph: self-loop";
      return GPEPS_ERR_ARG;
    }
    if (u > v) std::swap(u, v);
    if (seen.count({u, v})) {
      err = "graph: duplicate edge";
      return GPEPS_ERR_ARG;
    }
    seen[{u, v}] = e;
    t.ed[e] = {u, v};
  }
  t.inc.assign(g.n_nodes, {});
  for (int e = 0; e < g.n_edges; ++e) {
    t.inc[t.ed[e].first].push_back(e);
    t.inc[t.ed[e].second].push_back(e);
  }
  for (auto& l : t.inc)
    if ((int)l.size() > kMaxDeg) {
      err = "graph: vertex degree above 3 is not supported";
      return GPEPS_ERR_ARG;
    }
  if (g.colour) {
    t.colour.assign(g.colour, g.colour + g.n_edges);
  } else if (!kempe_colour(g.n_nodes, t.ed, t.colour, err)) {
    return GPEPS_ERR_ARG;
  }
  t.n_colours = 0;
  for (int e = 0; e < g.n_edges; ++e) {
    if (t.colour[e] < 0 || t.colour[e] > 63) {
      err = "graph: colour out of range 0..63";
      return GPEPS_ERR_ARG;
    }
    t.n_colours = std::max(t.n_colours, t.colour[e] + 1);
  }
  for (int v = 0; v < g.n_nodes; ++v)
    for (size_t a = 0; a < t.inc[v].size(); ++a)
      for (size_t b = a + 1; b < t.inc[v].size(); ++b)
        if (t.colour[t.inc[v][a]] == t.colour[t.inc[v][b]]) {
          err = "graph: colouring is not proper (two edges of one colour share a vertex)";
          return GPEPS_ERR_ARG;
        }
  return GPEPS_OK;
}

gpeps_status build_layout(const gpeps_graph* graphs, int32_t n_graphs, const int32_t* graph_of_instance,
                          int32_t n_instances, const gpeps_config* cfg, const double* theta_h, const double* theta_j,
                          Layout& L, std::string& err) {
  if (!graphs || n_graphs < 1 || !graph_of_instance || n_instances < 1 || !cfg) {
    err = "need >= 1 graph, >= 1 instance and a config";
    return GPEPS_ERR_ARG;
  }
  if (cfg->d_max < 1 || cfg->d_max > kMaxDBig) {
    err = "config: d_max must be in 1..64";
    return GPEPS_ERR_ARG;
  }
  if (cfg->d_max > kMaxD && cfg->adjoint) {
    err = "config: the adjoint supports d_max <= 32";
    return GPEPS_ERR_ARG;
  }
  if (cfg->d_max > kMaxD && cfg->trunc_rel < 1e-10) {
    err = "config: d_max > 32 needs trunc_rel >= 1e-10 (one singular-vector set is recovered through "
          "1/sigma, accurate to ~2^-52 sigma_0 / sigma)";
    return GPEPS_ERR_ARG;
  }
  if (cfg->precision != GPEPS_C64_F64SVD && cfg->precision != GPEPS_C128) {
    err = "config: unknown precision";
    return GPEPS_ERR_ARG;
  }
  if (!(cfg->trunc_rel >= 0.0) || !(cfg->trunc_rel < 1.0)) {
    err = "config: trunc_rel must be in [0, 1)";
    return GPEPS_ERR_ARG;
  }
  if (cfg->max_steps < 1) {
    err = "config: max_steps must be >= 1";
    return GPEPS_ERR_ARG;
  }
  if (cfg->adjoint < 0 || cfg->adjoint > 2) {
    err = "config: adjoint must be 0, 1 or 2";
    return GPEPS_ERR_ARG;
  }
  if (cfg->mode != GPEPS_MODE_BATCHED && cfg->mode != GPEPS_MODE_PLAIN) {
    err = "config: unknown mode";
    return GPEPS_ERR_ARG;
  }
  std::vector<GraphTables> gt(n_graphs);
  for (int g = 0; g < n_graphs; ++g) {
    gpeps_status s = check_graph(graphs[g], gt[g], err);
    if (s != GPEPS_OK) return s;
  }
  const int64_t D = cfg->d_max;
  const size_t esize = cfg->precision == GPEPS_C128 ? 16 : 8;
  L.n_classes = 0;
  for (int k = 0; k < n_instances; ++k) {
    const int g = graph_of_instance[k];
    if (g < 0 || g >= n_graphs) {
      err = "graph_of_instance: index out of range";
      return GPEPS_ERR_ARG;
    }
    L.n_classes = std::max(L.n_classes, gt[g].n_colours);
  }
  // vertices and edges of every instance
  int64_t goff = 0;
  L.inst_vert_begin.resize(n_instances);
  L.inst_vert_end.resize(n_instances);
  L.inst_edge_begin.resize(n_instances);
  L.inst_chunk_begin.resize(n_instances);
  L.inst_chunk_end.resize(n_instances);
  std::vector<int64_t> vgoff;
  for (int k = 0; k < n_instances; ++k) {
    const GraphTables& t = gt[graph_of_instance[k]];
    const int vb = L.NV, eb = L.NE;
    L.inst_vert_begin[k] = vb;
    L.inst_edge_begin[k] = eb;
    L.inst_chunk_begin[k] = (int)L.chunks.size();
    for (int v = 0; v < t.n_nodes; ++v) {
      VertexInfo vi{};
      const int deg = (int)t.inc[v].size();
      int64_t ps = 1;
      for (int l = 0; l < deg; ++l) ps *= D;
      vi.goff = goff;
      vi.deg = deg;
      vi.inst = k;
      for (int l = 0; l < kMaxDeg; ++l) vi.leg[l] = l < deg ? eb + t.inc[v][l] : -1;
      L.verts.push_back(vi);
      vgoff.push_back(goff);
      for (int64_t c = 0; c * 1024 < ps; ++c) L.chunks.push_back(((int64_t)(vb + v) << 32) | c);
      goff += 2 * ps;
    }
    L.inst_chunk_end[k] = (int)L.chunks.size();
    for (int e = 0; e < t.n_edges; ++e) {
      EdgeInfo ei{};
      ei.inst = k;
      const int ends[2] = {t.ed[e].first, t.ed[e].second};
      for (int sd = 0; sd < 2; ++sd) {
        const int v = ends[sd];
        const auto& legs = t.inc[v];
        const int deg = (int)legs.size();
        SideInfo& S = ei.side[sd];
        S.goff = vgoff[vb + v];
        int64_t ps = 1;
        for (int l = 0; l < deg; ++l) ps *= D;
        S.pstride = ps;
        S.deg = deg;
        S.oth[0] = S.oth[1] = -1;
        S.so[0] = S.so[1] = 0;
        int no = 0;
        for (int l = 0; l < deg; ++l) {
          int64_t stride = 1;
          for (int r = l + 1; r < deg; ++r) stride *= D;
          if (legs[l] == e) {
            S.sq = (int32_t)stride;
          } else {
            S.oth[no] = eb + legs[l];
            S.so[no] = (int32_t)stride;
            ++no;
          }
        }
      }
      L.edges.push_back(ei);
    }
    L.NV += t.n_nodes;
    L.NE += t.n_edges;
    L.inst_vert_end[k] = L.NV;
    InstParam ip{};
    const double th = theta_h ? theta_h[k] : 0.0;
    const double tj = theta_j ? theta_j[k] : 0.0;
    if (!std::isfinite(th) || !std::isfinite(tj)) {
      err = "theta_h / theta_j must be finite";
      return GPEPS_ERR_ARG;
    }
    ip.rx_c = std::cos(0.5 * th);
    ip.rx_s = std::sin(0.5 * th);
    ip.g_c = std::cos(0.5 * tj);
    ip.g_s = std::sin(0.5 * tj);
    L.inst.push_back(ip);
  }
  L.n_gamma = goff;
  // colour-class work lists: items instance by instance, in edge id order within an instance.
  // Workgroups go to the 8 XCDs round-robin by index, so item i runs on XCD i mod 8: with 48 edges
  // per class on the 127-qubit graph every instance spreads over all XCDs.  An (edge, instance)
  // order would send instances k = x (mod 8) to one XCD and unbalance a theta_h sweep, whose cost
  // grows with theta_h.  The instances go in descending |sin theta_h| (ties by index): a stronger
  // kick saturates the bonds sooner and makes every gate of the instance dearer, and launching
  // those items first keeps the longest ones off the tail of the launch.
  std::vector<int> inst_order(n_instances);
  for (int k = 0; k < n_instances; ++k) inst_order[k] = k;
  std::stable_sort(inst_order.begin(), inst_order.end(), [&](int a, int b) {
    const double ka = theta_h ? std::fabs(std::sin(theta_h[a])) : 0.0;
    const double kb = theta_h ? std::fabs(std::sin(theta_h[b])) : 0.0;
    return ka > kb;
  });
  L.class_begin.resize(L.n_classes);
  L.class_end.resize(L.n_classes);
  L.max_items = 0;
  for (int c = 0; c < L.n_classes; ++c) {
    L.class_begin[c] = (int)L.items.size();
    for (int k : inst_order) {
      const GraphTables& t = gt[graph_of_instance[k]];
      for (int e = 0; e < t.n_edges; ++e)
        if (t.colour[e] == c) L.items.push_back(L.inst_edge_begin[k] + e);
    }
    L.class_end[c] = (int)L.items.size();
    L.max_items = std::max(L.max_items, L.class_end[c] - L.class_begin[c]);
  }
  // end lists of the absorb, the re-absorb and the edge adjoint: the ends of a class whose site
  // has at most one other leg need one block of rows per slice, the others up to
  // D^2 / rows-per-block; the light ends are stored first, the launches take the heavy ones first
  L.rl_begin.resize(L.n_classes);
  L.rl_light.resize(L.n_classes);
  L.rl_heavy.resize(L.n_classes);
  for (int c = 0; c < L.n_classes; ++c) {
    L.rl_begin[c] = (int)L.rlist.size();
    for (int pass = 0; pass < 2; ++pass) {
      int n = 0;
      for (int it = L.class_begin[c]; it < L.class_end[c]; ++it)
        for (int sd = 0; sd < 2; ++sd)
          if ((L.edges[L.items[it]].side[sd].deg <= 2) == (pass == 0)) {
            L.rlist.push_back((it - L.class_begin[c]) * 2 + sd);
            ++n;
          }
      (pass == 0 ? L.rl_light : L.rl_heavy)[c] = n;
    }
  }
  const size_t slots = std::max(L.max_items, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max(bytes, size_t(1)));
    return o;
  };
  L.off_gamma = take((size_t)L.n_gamma * esize);
  L.off_lam = take((size_t)L.NE * D * sizeof(double));
  L.off_chi = take((size_t)L.NE * sizeof(int32_t));
  L.off_edges = take(L.edges.size() * sizeof(EdgeInfo));
  L.off_verts = take(L.verts.size() * sizeof(VertexInfo));
  // three parameter arrays: the instance angles, the same with negated sines (U^dagger), and
  // the identity gate (theta_J = 0) of the re-gauging sweeps
  L.off_inst = take(3 * L.inst.size() * sizeof(InstParam));
  L.off_items = take(L.items.size() * sizeof(int32_t));
  L.off_rlist = take(L.rlist.size() * sizeof(int32_t));
  // with the adjoint, the R factors, slot metadata and reverse-sweep buffers are kept for every
  // colour class of the step being reversed
  // (adjoint = 2: for every colour class of every step, so that the reverse sweep needs no recompute)
  const size_t ncl = cfg->adjoint ? (size_t)std::max(L.n_classes, 1) * (cfg->adjoint == 2 ? cfg->max_steps : 1) : 1;
  L.class_slots = slots;
  L.off_rbuf = take(ncl * slots * 4 * D * D * sizeof(double2));
  L.off_tbuf = take(slots * 4 * D * D * esize);
  L.off_stats = take(4 * sizeof(int64_t));
  L.off_meta = take(ncl * slots * sizeof(SlotMeta));
  L.off_z = take((size_t)L.NV * sizeof(double));
  L.off_hist = take((size_t)cfg->max_steps * L.NV * sizeof(double));
  L.off_ctr = take(4 * sizeof(int32_t));  // step counter, status word
  // belief-propagation messages: two buffers of one D x D float64 complex matrix per directed edge
  // (BP runs at d_max <= 32 only)
  L.off_bp = take(D <= kMaxD ? (size_t)2 * 2 * L.NE * D * D * sizeof(double2) : 0);
  // scratch of the two-site SVD for bond dimensions above 32 (Theta' and one vector set per item)
  L.off_big = take(D > kMaxD ? slots * (size_t)big_scratch((int)D) * sizeof(double2) : 0);
  L.off_bpres = take(sizeof(unsigned long long));
  L.off_chunks = take(L.chunks.size() * sizeof(int64_t));
  L.off_ivb = take(((size_t)n_instances + 1) * sizeof(int32_t));
  L.off_mean = take((size_t)n_instances * sizeof(double));
  if (cfg->adjoint) {
    // the state (site tensors, lambdas, bond dimensions) is the contiguous span gamma..chi
    L.state_bytes = L.off_chi + (size_t)L.NE * sizeof(int32_t) - L.off_gamma;
    L.state_slot = align_up(L.state_bytes);
    L.off_ckpt = take((size_t)cfg->max_steps * L.state_slot);
    L.off_snap = take((size_t)std::max(L.n_classes, 1) * (cfg->adjoint == 2 ? cfg->max_steps : 1) * L.state_slot);
    L.off_work = take(L.state_slot);
    L.off_gbar = take((size_t)L.n_gamma * sizeof(double2));
    L.off_lbar = take((size_t)L.NE * D * sizeof(double));
    L.off_thbar = take((size_t)n_instances * 2 * sizeof(double));
    L.off_dldz = take((size_t)L.NV * sizeof(double));
    L.off_bU = take(ncl * slots * 4 * D * D * sizeof(double2));
    L.off_bV = take(ncl * slots * 4 * D * D * sizeof(double2));
    L.off_bS = take(ncl * slots * 2 * D * sizeof(double));
    L.off_t64 = take(ncl * slots * 4 * D * D * sizeof(double2));
    L.off_wsb = take(slots * (size_t)adj_scratch((int)D) * sizeof(double2));
    L.off_ybuf = take(slots * 4 * D * D * sizeof(double2));
    L.off_ymode = take(slots * 4 * sizeof(int32_t));
    L.off_dldm = take((size_t)n_instances * sizeof(double));
    L.off_gpart = take(((size_t)L.NE + L.chunks.size()) * sizeof(double));
    L.off_wbar = take(slots * 4 * D * D * sizeof(double));
  }
  L.total = off;
  return GPEPS_OK;
}

}  // namespace

struct gpeps_ctx {
  std::string err;
  hipStream_t stream = nullptr;
  bool c128 = false;
  int D = 0, mode = 0, max_steps = 0, n_inst = 0;
  Layout L;
  DevState st{};
  const int32_t* d_items = nullptr;
  const int32_t* d_rlist = nullptr;
  int blocks_per_slice = 1;
  int steps_done = 0;
  hipGraphExec_t step_exec = nullptr;
  hipGraph_t step_graph = nullptr;
  hipGraphExec_t inv_exec = nullptr;  // the inverse step U^dagger, captured on first use
  hipGraph_t inv_graph = nullptr;
  bool adjoint = false;
  int adjoint_mode = 0;  // cfg.adjoint: 1 recompute each step in gpeps_backward, 2 keep every class's data
  char* ws = nullptr;
  std::vector<InstParam> inst_host;
  void* bp_scratch = nullptr;          // device address of the library's BP scratch array
  hipError_t bp_scratch_err = hipSuccess;  // status of its lookup on this context's device
};

namespace {

gpeps_status fail(gpeps_ctx* ctx, gpeps_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  g_thread_error = msg;
  return s;
}

#define HIP_TRY(ctx, call)                                                                          \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess)                                                                           \
      return fail((ctx), GPEPS_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

// Launch one kind of edge kernel over a range of items, in the context's mode.
// The view with the row-block work list of the colour class when [first, first + count) is a
// whole class (a launch over part of a class keeps the full grid).
DevState with_rows(const gpeps_ctx* c, DevState v, int first, int count) {
  const Layout& L = c->L;
  v.rlist = nullptr;
  v.rl_light = v.rl_heavy = 0;
  for (int cl = 0; cl < L.n_classes; ++cl)
    if (L.class_begin[cl] == first && L.class_end[cl] - first == count) {
      v.rlist = c->d_rlist + L.rl_begin[cl];
      v.rl_light = L.rl_light[cl];
      v.rl_heavy = L.rl_heavy[cl];
    }
  return v;
}

gpeps_status enqueue_edge_kernel(gpeps_ctx* c, int which, int first, int count, hipEvent_t* ev, int* nev) {
  (void)ev;
  (void)nev;
  HIP_TRY(c, launch_edge_kernel(which, c->c128, with_rows(c, c->st, first, count), c->d_items, first, count,
                                c->blocks_per_slice, c->stream));
  return GPEPS_OK;
}

struct Timer {
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;
};

gpeps_status timed(gpeps_ctx* c, Timer* tm, int kind, hipEvent_t& start) {
  if (!tm || !tm->on) return GPEPS_OK;
  HIP_TRY(c, hipEventCreate(&start));
  HIP_TRY(c, hipEventRecord(start, c->stream));
  return GPEPS_OK;
}

gpeps_status timed_end(gpeps_ctx* c, Timer* tm, int kind, hipEvent_t start) {
  if (!tm || !tm->on) return GPEPS_OK;
  hipEvent_t stop;
  HIP_TRY(c, hipEventCreate(&stop));
  HIP_TRY(c, hipEventRecord(stop, c->stream));
  tm->ev.push_back(start);
  tm->ev.push_back(stop);
  tm->kind.push_back(kind);
  return GPEPS_OK;
}

// RX layer over all instances (batched) or instance by instance (plain).
// The three parameter arrays: the angles, those of U(theta)^dagger (RX(-theta_h) and RZZ(-theta_J)
// flip the sines only), and the identity gate (cos 0, sin 0) of the re-gauging sweeps.
std::vector<InstParam> with_inverse(const std::vector<InstParam>& fwd) {
  std::vector<InstParam> v(fwd);
  for (const InstParam& p : fwd) v.push_back(InstParam{p.rx_c, -p.rx_s, p.g_c, -p.g_s});
  for (size_t k = 0; k < fwd.size(); ++k) v.push_back(InstParam{1.0, 0.0, 1.0, 0.0});
  return v;
}


// The RX layer; `advance` (a recorded step: the readout that closes it writes history row
// counter - 1) makes its first launch advance the device step counter.
gpeps_status enqueue_rx(gpeps_ctx* c, Timer* tm, int advance) {
  const Layout& L = c->L;
  if (c->mode == GPEPS_MODE_BATCHED) {
    hipEvent_t s0 = nullptr;
    gpeps_status s = timed(c, tm, 0, s0);
    if (s) return s;
    HIP_TRY(c, launch_rx(c->c128, c->st, 0, (int)L.chunks.size(), advance, c->stream));
    return timed_end(c, tm, 0, s0);
  }
  int adv = advance;  // the first launch with chunks advances the counter
  for (int k = 0; k < c->n_inst; ++k) {
    hipEvent_t s0 = nullptr;
    gpeps_status s = timed(c, tm, 0, s0);
    if (s) return s;
    const int n = L.inst_chunk_end[k] - L.inst_chunk_begin[k];
    HIP_TRY(c, launch_rx(c->c128, c->st, L.inst_chunk_begin[k], n, adv, c->stream));
    if (n > 0) adv = 0;
    s = timed_end(c, tm, 0, s0);
    if (s) return s;
  }
  return GPEPS_OK;
}

gpeps_status enqueue_rzz(gpeps_ctx* c, Timer* tm) {
  const Layout& L = c->L;
  for (int cl = 0; cl < L.n_classes; ++cl) {
    const int b = L.class_begin[cl], e = L.class_end[cl];
    if (c->mode == GPEPS_MODE_BATCHED) {
      for (int which = 1; which <= 3; ++which) {
        hipEvent_t s0 = nullptr;
        gpeps_status s = timed(c, tm, which, s0);
        if (s) return s;
        s = enqueue_edge_kernel(c, which, b, e - b, nullptr, nullptr);
        if (s) return s;
        s = timed_end(c, tm, which, s0);
        if (s) return s;
      }
    } else {
      for (int it = b; it < e; ++it)
        for (int which = 1; which <= 3; ++which) {
          hipEvent_t s0 = nullptr;
          gpeps_status s = timed(c, tm, which, s0);
          if (s) return s;
          s = enqueue_edge_kernel(c, which, it, 1, nullptr, nullptr);
          if (s) return s;
          s = timed_end(c, tm, which, s0);
          if (s) return s;
        }
    }
  }
  return GPEPS_OK;
}

gpeps_status enqueue_readout(gpeps_ctx* c, int record, Timer* tm) {
  const Layout& L = c->L;
  if (c->mode == GPEPS_MODE_BATCHED) {
    hipEvent_t s0 = nullptr;
    gpeps_status s = timed(c, tm, 4, s0);
    if (s) return s;
    HIP_TRY(c, launch_expect_z(c->c128, c->st, 0, L.NV, record ? 1 : 0, c->stream));
    return timed_end(c, tm, 4, s0);
  } else {
    for (int k = 0; k < c->n_inst; ++k) {
      hipEvent_t s0 = nullptr;
      gpeps_status s = timed(c, tm, 4, s0);
      if (s) return s;
      HIP_TRY(c, launch_expect_z(c->c128, c->st, L.inst_vert_begin[k], L.inst_vert_end[k] - L.inst_vert_begin[k],
                                 record, c->stream));
      s = timed_end(c, tm, 4, s0);
      if (s) return s;
    }
  }
  return GPEPS_OK;
}

// DevState whose state pointers (gamma, lambda, bond dims) point into a state copy at `base`.
// The per-class buffers of colour class cl (R factors, slot metadata, reverse-sweep triplets).
// The per-slot buffers (R factors, metadata, triplets, float64 T) advanced by `sl` slots.
DevState slot_view(const gpeps_ctx* c, DevState v, int64_t sl) {
  const int64_t q = (int64_t)c->D * c->D;
  v.rbuf += sl * 4 * q;
  v.meta += sl;
  v.bU += sl * 4 * q;
  v.bV += sl * 4 * q;
  v.bS += sl * 2 * c->D;
  v.t64 += sl * 4 * q;
  return v;
}

DevState class_view(const gpeps_ctx* c, DevState v, int cl) {
  const int64_t q = (int64_t)c->D * c->D;
  const int64_t sl = (int64_t)c->L.class_slots * cl;
  v.rbuf += sl * 4 * q;
  v.meta += sl;
  v.bU += sl * 4 * q;
  v.bV += sl * 4 * q;
  v.bS += sl * 2 * c->D;
  v.t64 += sl * 4 * q;
  return v;
}

DevState state_view(const gpeps_ctx* c, char* base) {
  DevState v = c->st;
  const Layout& L = c->L;
  v.gamma = base;
  v.lam = reinterpret_cast<double*>(base + (L.off_lam - L.off_gamma));
  v.chi = reinterpret_cast<int32_t*>(base + (L.off_chi - L.off_gamma));
  return v;
}

// cfg.adjoint = 2: one forward step that keeps, for each colour class, the state before the class
// (snapshot t C + cl) and the update's R factors, metadata, singular triplets and float64 T (class
// buffers t C + cl), computed by the same SVD kernel the reverse sweep's recompute runs.  t is the
// step's index in the history.
gpeps_status enqueue_rzz_stored(gpeps_ctx* c, Timer* tm) {
  const Layout& L = c->L;
  const int C = L.n_classes, t = c->steps_done;
  for (int cl = 0; cl < C; ++cl) {
    char* sn = c->ws + L.off_snap + (size_t)(t * C + cl) * L.state_slot;
    HIP_TRY(c, hipMemcpyAsync(sn, c->ws + L.off_gamma, L.state_bytes, hipMemcpyDeviceToDevice, c->stream));
    const DevState sc = class_view(c, c->st, t * C + cl);
    const int b = L.class_begin[cl], e = L.class_end[cl];
    const bool batched = c->mode == GPEPS_MODE_BATCHED;
    for (int it = b; it < e; it += batched ? (e - b) : 1) {
      const int n = batched ? e - b : 1;
      // a one-item launch works in slot 0: point it at the item's slot of the class, where the
      // reverse sweep (launched over the whole class) looks for it
      const DevState si = batched ? sc : slot_view(c, sc, it - b);
      for (int which = 1; which <= 3; ++which) {
        hipEvent_t s0 = nullptr;
        gpeps_status s = timed(c, tm, which, s0);
        if (s) return s;
        if (which == 2) HIP_TRY(c, launch_svd_bwd(c->c128, si, c->d_items, it, n, c->stream));
        else HIP_TRY(c, launch_edge_kernel(which, c->c128, with_rows(c, si, it, n), c->d_items, it, n, c->blocks_per_slice,
                                           c->stream));
        s = timed_end(c, tm, which, s0);
        if (s) return s;
      }
    }
  }
  return GPEPS_OK;
}

gpeps_status enqueue_step(gpeps_ctx* c, Timer* tm) {
  if (c->adjoint) {
    const Layout& L = c->L;
    HIP_TRY(c, launch_checkpoint(c->st, c->ws + L.off_gamma, c->ws + L.off_ckpt, (int64_t)L.state_bytes,
                                 (int64_t)L.state_slot, c->stream));
  }
  gpeps_status s = enqueue_rx(c, tm, 1);
  if (s) return s;
  s = c->adjoint_mode == 2 ? enqueue_rzz_stored(c, tm) : enqueue_rzz(c, tm);
  if (s) return s;
  return enqueue_readout(c, 1, tm);
}

// One re-gauging sweep: the simple update with the identity gate on every edge, class by class.
// The state is unchanged up to singular values under the cutoff; the fixed point of the sweeps
// is the fixed point of belief propagation (BP gauging).
gpeps_status enqueue_regauge(gpeps_ctx* c) {
  const InstParam* fwd = c->st.inst;
  c->st.inst = fwd + 2 * c->n_inst;
  gpeps_status s = enqueue_rzz(c, nullptr);
  c->st.inst = fwd;
  return s;
}

// U(theta)^dagger (Appendix B): the RZZ layer, class by class in the forward order, then the RX
// layer, both reading the second parameter array; then the readout into the next history row.
gpeps_status enqueue_inverse_step(gpeps_ctx* c) {
  const InstParam* fwd = c->st.inst;
  c->st.inst = fwd + c->n_inst;
  gpeps_status s = enqueue_rzz(c, nullptr);
  if (s == GPEPS_OK) s = enqueue_rx(c, nullptr, 1);
  c->st.inst = fwd;
  if (s) return s;
  return enqueue_readout(c, 1, nullptr);
}

gpeps_status ensure_inverse_graph(gpeps_ctx* c) {
  if (c->inv_exec) return GPEPS_OK;
  HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  gpeps_status s = enqueue_inverse_step(c);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &graph);
  if (s != GPEPS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return fail(c, GPEPS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  c->inv_graph = graph;
  HIP_TRY(c, hipGraphInstantiate(&c->inv_exec, graph, nullptr, nullptr, 0));
  return GPEPS_OK;
}

gpeps_status ensure_step_graph(gpeps_ctx* c) {
  if (c->step_exec) return GPEPS_OK;
  HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  gpeps_status s = enqueue_step(c, nullptr);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &graph);
  if (s != GPEPS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return fail(c, GPEPS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  c->step_graph = graph;
  HIP_TRY(c, hipGraphInstantiate(&c->step_exec, graph, nullptr, nullptr, 0));
  return GPEPS_OK;
}

gpeps_status check_status_word(gpeps_ctx* c) {
  int32_t word = 0;
  HIP_TRY(c, hipMemcpyAsync(&word, c->st.status, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (word) {
    std::string m = "device status word:";
    if (word & kStatusNonFinite) m += " non-finite value;";
    if (word & kStatusNoConverge) m += " Jacobi SVD did not converge within max_jacobi_sweeps;";
    if (word & kStatusZeroTheta) m += " two-site tensor is zero;";
    return fail(c, GPEPS_ERR_NUMERIC, m);
  }
  return GPEPS_OK;
}

gpeps_status reverse_sweep(gpeps_ctx* c, double* dtheta_h, double* dtheta_j, Timer* tm);

}  // namespace

extern "C" {

gpeps_status gpeps_workspace_size(const gpeps_graph* graphs, int32_t n_graphs, const int32_t* graph_of_instance,
                                  int32_t n_instances, const gpeps_config* cfg, size_t* bytes) {
  if (!bytes) return fail(nullptr, GPEPS_ERR_ARG, "bytes is NULL");
  Layout L;
  std::string err;
  gpeps_status s = build_layout(graphs, n_graphs, graph_of_instance, n_instances, cfg, nullptr, nullptr, L, err);
  if (s != GPEPS_OK) return fail(nullptr, s, err);
  *bytes = L.total;
  return GPEPS_OK;
}

gpeps_status gpeps_init(gpeps_ctx** out, const gpeps_graph* graphs, int32_t n_graphs,
                        const int32_t* graph_of_instance, int32_t n_instances, const double* theta_h,
                        const double* theta_j, const gpeps_config* cfg, void* d_workspace, size_t ws_bytes,
                        void* hip_stream) {
  if (!out) return fail(nullptr, GPEPS_ERR_ARG, "ctx pointer is NULL");
  *out = nullptr;
  if (!theta_h || !theta_j) return fail(nullptr, GPEPS_ERR_ARG, "theta_h and theta_j are required");
  gpeps_ctx* c = new gpeps_ctx();
  std::string err;
  gpeps_status s = build_layout(graphs, n_graphs, graph_of_instance, n_instances, cfg, theta_h, theta_j, c->L, err);
  if (s != GPEPS_OK) {
    delete c;
    return fail(nullptr, s, err);
  }
  if (!d_workspace || ws_bytes < c->L.total || (reinterpret_cast<uintptr_t>(d_workspace) & 255)) {
    const size_t need = c->L.total;
    delete c;
    return fail(nullptr, GPEPS_ERR_WORKSPACE,
                "workspace missing, misaligned or too small (need " + std::to_string(need) + " bytes)");
  }
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->c128 = cfg->precision == GPEPS_C128;
  c->D = cfg->d_max;
  c->mode = cfg->mode;
  c->max_steps = cfg->max_steps;
  c->n_inst = n_instances;
  int max_rows = 1;
  for (int l = 0; l < kMaxDeg - 1; ++l) max_rows *= c->D;
  c->blocks_per_slice = (max_rows + kRowBlock - 1) / kRowBlock;
  const Layout& L = c->L;
  char* ws = static_cast<char*>(d_workspace);
  DevState& st = c->st;
  st.gamma = ws + L.off_gamma;
  st.lam = reinterpret_cast<double*>(ws + L.off_lam);
  st.chi = reinterpret_cast<int32_t*>(ws + L.off_chi);
  st.edges = reinterpret_cast<const EdgeInfo*>(ws + L.off_edges);
  st.verts = reinterpret_cast<const VertexInfo*>(ws + L.off_verts);
  st.inst = reinterpret_cast<const InstParam*>(ws + L.off_inst);
  c->d_items = reinterpret_cast<const int32_t*>(ws + L.off_items);
  c->d_rlist = reinterpret_cast<const int32_t*>(ws + L.off_rlist);
  st.rbuf = reinterpret_cast<double2*>(ws + L.off_rbuf);
  st.tbuf = ws + L.off_tbuf;
  st.stats = reinterpret_cast<int64_t*>(ws + L.off_stats);
  st.meta = reinterpret_cast<SlotMeta*>(ws + L.off_meta);
  st.z = reinterpret_cast<double*>(ws + L.off_z);
  st.hist = reinterpret_cast<double*>(ws + L.off_hist);
  st.step_ctr = reinterpret_cast<int32_t*>(ws + L.off_ctr);
  st.bp_msg = reinterpret_cast<double2*>(ws + L.off_bp);
  st.bp_res = reinterpret_cast<unsigned long long*>(ws + L.off_bpres);
  st.status = st.step_ctr + 1;
  st.chunks = reinterpret_cast<const int64_t*>(ws + L.off_chunks);
  st.inst_vb = reinterpret_cast<const int32_t*>(ws + L.off_ivb);
  st.big = c->D > kMaxD ? reinterpret_cast<double2*>(ws + L.off_big) : nullptr;
  st.mean = reinterpret_cast<double*>(ws + L.off_mean);
  st.n_inst = n_instances;
  c->ws = ws;
  c->adjoint = cfg->adjoint != 0;
  c->adjoint_mode = cfg->adjoint;
  c->inst_host = L.inst;
  if (c->adjoint) {
    st.gbar = reinterpret_cast<double2*>(ws + L.off_gbar);
    st.lbar = reinterpret_cast<double*>(ws + L.off_lbar);
    st.thbar = reinterpret_cast<double*>(ws + L.off_thbar);
    st.dldz = reinterpret_cast<const double*>(ws + L.off_dldz);
    st.bU = reinterpret_cast<double2*>(ws + L.off_bU);
    st.bV = reinterpret_cast<double2*>(ws + L.off_bV);
    st.bS = reinterpret_cast<double*>(ws + L.off_bS);
    st.t64 = reinterpret_cast<double2*>(ws + L.off_t64);
    st.wsb = reinterpret_cast<double2*>(ws + L.off_wsb);
    st.ymode = reinterpret_cast<int32_t*>(ws + L.off_ymode);
    st.dldm = reinterpret_cast<const double*>(ws + L.off_dldm);
    st.gpart = reinterpret_cast<double*>(ws + L.off_gpart);
    st.wbar = reinterpret_cast<double*>(ws + L.off_wbar);
  }
  st.D = c->D;
  st.NV = L.NV;
  st.NE = L.NE;
  st.max_sweeps = cfg->max_jacobi_sweeps > 0 ? cfg->max_jacobi_sweeps : 40;
  st.max_steps = cfg->max_steps;
  st.trunc_rel = cfg->trunc_rel;
  st.tune_rb = 2;
  st.tune_qr = 16;
  st.tune_svd = 256;
  // site tensors larger than the 256 MB last-level cache are streamed past the caches by the
  // re-absorb; a state that fits stays cached for the readout and the next gate (measured: a
  // 150 MiB state ran slower streamed, 620 and 665 MiB ones faster)
  st.stream_gamma = (size_t)L.n_gamma * (c->c128 ? sizeof(double2) : sizeof(float2)) > ((size_t)256 << 20) ? 1 : 0;
  auto h2d = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, c->stream);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = h2d(L.off_edges, L.edges.data(), L.edges.size() * sizeof(EdgeInfo));
  if (e == hipSuccess) e = h2d(L.off_verts, L.verts.data(), L.verts.size() * sizeof(VertexInfo));
  const std::vector<InstParam> both = with_inverse(L.inst);
  if (e == hipSuccess) e = h2d(L.off_inst, both.data(), both.size() * sizeof(InstParam));
  if (e == hipSuccess) e = h2d(L.off_items, L.items.data(), L.items.size() * sizeof(int32_t));
  if (e == hipSuccess) e = h2d(L.off_rlist, L.rlist.data(), L.rlist.size() * sizeof(int32_t));
  if (e == hipSuccess) e = h2d(L.off_chunks, L.chunks.data(), L.chunks.size() * sizeof(int64_t));
  std::vector<int32_t> ivb(L.inst_vert_begin.begin(), L.inst_vert_begin.end());
  ivb.push_back(L.NV);
  if (e == hipSuccess) e = h2d(L.off_ivb, ivb.data(), ivb.size() * sizeof(int32_t));
  // the device address of the BP scratch array of gpeps_bp_expect_z_noalloc, looked up once per
  // device; a failed lookup only disables that call
  c->bp_scratch_err = bp_scratch_address(&c->bp_scratch);
  if (e == hipSuccess) e = launch_reset(c->c128, st, L.n_gamma, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    const std::string m = std::string("gpeps_init: ") + hipGetErrorString(e);
    delete c;
    return fail(nullptr, GPEPS_ERR_HIP, m);
  }
  *out = c;
  return GPEPS_OK;
}

gpeps_status gpeps_reset(gpeps_ctx* c) {
  if (!c) return fail(nullptr, GPEPS_ERR_ARG, "ctx is NULL");
  HIP_TRY(c, launch_reset(c->c128, c->st, c->L.n_gamma, c->stream));
  c->steps_done = 0;
  return GPEPS_OK;
}

gpeps_status gpeps_apply_layer(gpeps_ctx* c, int32_t kind, int32_t repeat) {
  if (!c) return fail(nullptr, GPEPS_ERR_ARG, "ctx is NULL");
  if (repeat < 0) return fail(c, GPEPS_ERR_ARG, "repeat must be >= 0");
  if (kind != GPEPS_LAYER_RX && kind != GPEPS_LAYER_RZZ && kind != GPEPS_STEP && kind != GPEPS_STEP_INVERSE &&
      kind != GPEPS_LAYER_REGAUGE)
    return fail(c, GPEPS_ERR_ARG, "unknown layer kind");
  const bool records = kind == GPEPS_STEP || kind == GPEPS_STEP_INVERSE;
  if (kind == GPEPS_STEP_INVERSE && c->adjoint)
    return fail(c, GPEPS_ERR_STATE, "GPEPS_STEP_INVERSE is not recorded for the adjoint (context has cfg.adjoint = 1)");
  if (kind == GPEPS_LAYER_REGAUGE && c->adjoint)
    return fail(c, GPEPS_ERR_STATE, "GPEPS_LAYER_REGAUGE is not recorded for the adjoint (context has cfg.adjoint = 1)");
  if ((kind == GPEPS_LAYER_RX || kind == GPEPS_LAYER_RZZ) && c->adjoint)
    return fail(c, GPEPS_ERR_STATE,
                "single layers are not checkpointed for the adjoint (context has cfg.adjoint != 0): use GPEPS_STEP");
  if (records && c->steps_done + repeat > c->max_steps)
    return fail(c, GPEPS_ERR_STATE, "history full: cfg.max_steps steps already recorded (call gpeps_reset)");
  for (int r = 0; r < repeat; ++r) {
    gpeps_status s = GPEPS_OK;
    if (kind == GPEPS_LAYER_RX) {
      s = enqueue_rx(c, nullptr, 0);
    } else if (kind == GPEPS_LAYER_RZZ) {
      s = enqueue_rzz(c, nullptr);
    } else if (kind == GPEPS_LAYER_REGAUGE) {
      s = enqueue_regauge(c);
    } else if (kind == GPEPS_STEP_INVERSE) {
      if (c->mode == GPEPS_MODE_BATCHED && c->stream != nullptr) {
        s = ensure_inverse_graph(c);
        if (s == GPEPS_OK) {
          hipError_t e = hipGraphLaunch(c->inv_exec, c->stream);
          if (e != hipSuccess) s = fail(c, GPEPS_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        }
      } else {
        s = enqueue_inverse_step(c);
      }
    } else if (c->mode == GPEPS_MODE_BATCHED && c->stream != nullptr && c->adjoint_mode != 2) {
      s = ensure_step_graph(c);
      if (s == GPEPS_OK) {
        hipError_t e = hipGraphLaunch(c->step_exec, c->stream);
        if (e != hipSuccess) s = fail(c, GPEPS_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
      }
    } else {
      s = enqueue_step(c, nullptr);
    }
    if (s != GPEPS_OK) return s;
    if (records) c->steps_done++;
  }
  return GPEPS_OK;
}

gpeps_status gpeps_expect_z(gpeps_ctx* c, double* out, int32_t out_on_device) {
  if (!c || !out) return fail(c, GPEPS_ERR_ARG, "ctx and out are required");
  gpeps_status s = enqueue_readout(c, 0, nullptr);
  if (s) return s;
  const size_t bytes = (size_t)c->L.NV * sizeof(double);
  if (out_on_device) {
    HIP_TRY(c, hipMemcpyAsync(out, c->st.z, bytes, hipMemcpyDeviceToDevice, c->stream));
    return GPEPS_OK;
  }
  HIP_TRY(c, hipMemcpyAsync(out, c->st.z, bytes, hipMemcpyDeviceToHost, c->stream));
  return check_status_word(c);
}

gpeps_status gpeps_bp_expect_z(gpeps_ctx* c, int32_t iters, double* out, int32_t out_on_device, double* residual) {
  if (!c || !out) return fail(c, GPEPS_ERR_ARG, "ctx and out are required");
  if (c->D > kMaxD) return fail(c, GPEPS_ERR_ARG, "belief propagation supports d_max <= 32");
  if (iters < 0 || iters > 100000) return fail(c, GPEPS_ERR_ARG, "iters must be in 0..100000");
  HIP_TRY(c, launch_bp(c->c128, c->st, iters, c->stream));
  const size_t bytes = (size_t)c->L.NV * sizeof(double);
  HIP_TRY(c, hipMemcpyAsync(out, c->st.z, bytes, out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            c->stream));
  if (residual) {
    unsigned long long bits = 0;
    HIP_TRY(c, hipMemcpyAsync(&bits, c->st.bp_res, sizeof(bits), hipMemcpyDeviceToHost, c->stream));
    gpeps_status s = check_status_word(c);
    double r = 0.0;
    std::memcpy(&r, &bits, sizeof(r));
    // with no edges no message exists (and the residual word was never written)
    *residual = (iters > 0 && c->L.NE > 0) ? r : 0.0;
    return s;
  }
  return out_on_device ? GPEPS_OK : check_status_word(c);
}

gpeps_status gpeps_bp_expect_z_noalloc(gpeps_ctx* c, int32_t iters, double* out, int32_t out_on_device,
                                       double* residual) {
  if (!c || !out) return fail(c, GPEPS_ERR_ARG, "ctx and out are required");
  if (c->D > kMaxD) return fail(c, GPEPS_ERR_ARG, "belief propagation supports d_max <= 32");
  if (iters < 0 || iters > 100000) return fail(c, GPEPS_ERR_ARG, "iters must be in 0..100000");
  if (c->bp_scratch_err != hipSuccess || !c->bp_scratch)
    return fail(c, GPEPS_ERR_HIP, std::string("BP scratch array unavailable on this device: ") +
                                      hipGetErrorString(c->bp_scratch_err));
  const size_t msg_bytes = (size_t)2 * 2 * c->L.NE * c->D * c->D * sizeof(double2);
  if (msg_bytes + 256 > kBpScratchBytes)
    return fail(c, GPEPS_ERR_ARG,
                "BP messages need " + std::to_string(msg_bytes + 256) + " bytes, more than the " +
                    std::to_string(kBpScratchBytes) + "-byte device scratch of gpeps_bp_expect_z_noalloc "
                    "(use gpeps_bp_expect_z)");
  DevState sv = c->st;
  sv.bp_msg = reinterpret_cast<double2*>(c->bp_scratch);
  sv.bp_res = reinterpret_cast<unsigned long long*>(static_cast<char*>(c->bp_scratch) + align_up(msg_bytes));
  HIP_TRY(c, launch_bp(c->c128, sv, iters, c->stream));
  const size_t bytes = (size_t)c->L.NV * sizeof(double);
  HIP_TRY(c, hipMemcpyAsync(out, c->st.z, bytes, out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            c->stream));
  if (residual) {
    unsigned long long bits = 0;
    HIP_TRY(c, hipMemcpyAsync(&bits, sv.bp_res, sizeof(bits), hipMemcpyDeviceToHost, c->stream));
    gpeps_status s = check_status_word(c);
    double r = 0.0;
    std::memcpy(&r, &bits, sizeof(r));
    *residual = (iters > 0 && c->L.NE > 0) ? r : 0.0;
    return s;
  }
  return out_on_device ? GPEPS_OK : check_status_word(c);
}

gpeps_status gpeps_z_history(gpeps_ctx* c, double* out, int32_t out_on_device, int32_t* steps_done) {
  if (!c) return fail(nullptr, GPEPS_ERR_ARG, "ctx is NULL");
  if (steps_done) *steps_done = c->steps_done;
  if (!out || c->steps_done == 0) return GPEPS_OK;
  const size_t bytes = (size_t)c->steps_done * c->L.NV * sizeof(double);
  if (out_on_device) {
    HIP_TRY(c, hipMemcpyAsync(out, c->st.hist, bytes, hipMemcpyDeviceToDevice, c->stream));
    return GPEPS_OK;
  }
  HIP_TRY(c, hipMemcpyAsync(out, c->st.hist, bytes, hipMemcpyDeviceToHost, c->stream));
  return check_status_word(c);
}

gpeps_status gpeps_bond_dims(gpeps_ctx* c, int32_t* out) {
  if (!c || !out) return fail(c, GPEPS_ERR_ARG, "ctx and out are required");
  HIP_TRY(c, hipMemcpyAsync(out, c->st.chi, (size_t)c->L.NE * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  return check_status_word(c);
}

gpeps_status gpeps_set_angles(gpeps_ctx* c, const double* theta_h, const double* theta_j) {
  if (!c || !theta_h || !theta_j) return fail(c, GPEPS_ERR_ARG, "ctx, theta_h and theta_j are required");
  if (c->adjoint && c->steps_done > 0)
    return fail(c, GPEPS_ERR_STATE,
                "the adjoint differentiates the recorded steps at their angles: call gpeps_reset before gpeps_set_angles");
  for (int k = 0; k < c->n_inst; ++k) {
    if (!std::isfinite(theta_h[k]) || !std::isfinite(theta_j[k]))
      return fail(c, GPEPS_ERR_ARG, "theta_h / theta_j must be finite");
    c->inst_host[k].rx_c = std::cos(0.5 * theta_h[k]);
    c->inst_host[k].rx_s = std::sin(0.5 * theta_h[k]);
    c->inst_host[k].g_c = std::cos(0.5 * theta_j[k]);
    c->inst_host[k].g_s = std::sin(0.5 * theta_j[k]);
  }
  const std::vector<InstParam> both = with_inverse(c->inst_host);
  HIP_TRY(c, hipMemcpyAsync(c->ws + c->L.off_inst, both.data(), both.size() * sizeof(InstParam), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return GPEPS_OK;
}

gpeps_status gpeps_backward(gpeps_ctx* c, const double* dl_dz, int32_t dl_dz_on_device, double* dtheta_h,
                            double* dtheta_j) {
  if (!c || !dl_dz) return fail(c, GPEPS_ERR_ARG, "ctx and dl_dz are required");
  if (!c->adjoint) return fail(c, GPEPS_ERR_STATE, "context was created with cfg.adjoint = 0");
  if (c->steps_done < 1) return fail(c, GPEPS_ERR_STATE, "no Trotter step recorded: run GPEPS_STEP first");
  HIP_TRY(c, hipMemcpyAsync(c->ws + c->L.off_dldz, dl_dz, (size_t)c->L.NV * sizeof(double),
                            dl_dz_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  return reverse_sweep(c, dtheta_h, dtheta_j, nullptr);
}

gpeps_status gpeps_mean_z(gpeps_ctx* c, double* out, int32_t out_on_device) {
  if (!c || !out) return fail(c, GPEPS_ERR_ARG, "ctx and out are required");
  if (c->steps_done < 1) return fail(c, GPEPS_ERR_STATE, "no <Z> row recorded: run GPEPS_STEP first");
  HIP_TRY(c, launch_mean_z(c->st, c->steps_done - 1, c->stream));
  const size_t bytes = (size_t)c->n_inst * sizeof(double);
  HIP_TRY(c, hipMemcpyAsync(out, c->st.mean, bytes, out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            c->stream));
  return out_on_device ? GPEPS_OK : check_status_word(c);
}

gpeps_status gpeps_backward_mean_z(gpeps_ctx* c, const double* dl_dm, double* dtheta_h, double* dtheta_j) {
  if (!c || !dl_dm) return fail(c, GPEPS_ERR_ARG, "ctx and dl_dm are required");
  if (!c->adjoint) return fail(c, GPEPS_ERR_STATE, "context was created with cfg.adjoint = 0");
  if (c->steps_done < 1) return fail(c, GPEPS_ERR_STATE, "no Trotter step recorded: run GPEPS_STEP first");
  for (int k = 0; k < c->n_inst; ++k)
    if (!std::isfinite(dl_dm[k])) return fail(c, GPEPS_ERR_ARG, "dl_dm must be finite");
  HIP_TRY(c, hipMemcpyAsync(c->ws + c->L.off_dldm, dl_dm, (size_t)c->n_inst * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, launch_seed_mean(c->st, c->stream));
  return reverse_sweep(c, dtheta_h, dtheta_j, nullptr);
}

}  // extern "C"

namespace {

// Kernel kinds of the reverse sweep timed by gpeps_time_backward.
constexpr int kAdjKinds = 9;
const char* const kAdjKindNames[kAdjKinds] = {"recompute_absorb", "recompute_theta_svd", "recompute_reabsorb",
                                              "adj_tbar", "adj_small", "adj_rows", "adj_rx", "adj_readout",
                                              "adj_lbar"};

#define TIMED_LAUNCH(kind, call)                       \
  do {                                                 \
    hipEvent_t ev_ = nullptr;                          \
    gpeps_status s_ = timed(c, tm, (kind), ev_);       \
    if (s_ != GPEPS_OK) return s_;                     \
    HIP_TRY(c, call);                                  \
    s_ = timed_end(c, tm, (kind), ev_);                \
    if (s_ != GPEPS_OK) return s_;                     \
  } while (0)

// The reverse sweep of every recorded step, seeded by dL/d<Z_v> already in the dl_dz buffer.
// tm (may be NULL) receives an event pair around every kernel launch.
gpeps_status reverse_sweep(gpeps_ctx* c, double* dtheta_h, double* dtheta_j, Timer* tm) {
  const Layout& L = c->L;
  DevState& st = c->st;
  HIP_TRY(c, launch_fill_d(reinterpret_cast<double*>(st.gbar), L.n_gamma * 2, c->stream));
  HIP_TRY(c, launch_fill_d(st.lbar, (int64_t)L.NE * c->D, c->stream));
  HIP_TRY(c, launch_fill_d(st.thbar, (int64_t)c->n_inst * 2, c->stream));
  HIP_TRY(c, launch_fill_d(st.gpart, (int64_t)L.NE + (int64_t)L.chunks.size(), c->stream));
  TIMED_LAUNCH(7, launch_adjoint(4, c->c128, st, c->d_items, 0, 0, c->blocks_per_slice, nullptr, c->stream));
  char* work = c->ws + L.off_work;
  const DevState sw = state_view(c, work);
  const int C = L.n_classes;
  const bool stored = c->adjoint_mode == 2;
  for (int t = c->steps_done - 1; t >= 0; --t) {
    char* ck = c->ws + L.off_ckpt + (size_t)t * L.state_slot;
    // buffers of step t: kept by the forward pass (adjoint = 2), else recomputed into the
    // per-class buffers 0..C-1
    const int cb = stored ? t * C : 0;
    if (!stored) {
      HIP_TRY(c, hipMemcpyAsync(work, ck, L.state_bytes, hipMemcpyDeviceToDevice, c->stream));
      HIP_TRY(c, launch_rx(c->c128, sw, 0, (int)L.chunks.size(), 0, c->stream));
      // recompute the step: the state before each class is saved, and each class's update keeps
      // its R factors, metadata, singular triplets and float64 T in that class's buffers
      for (int cl = 0; cl < C; ++cl) {
        char* sn = c->ws + L.off_snap + (size_t)cl * L.state_slot;
        HIP_TRY(c, hipMemcpyAsync(sn, work, L.state_bytes, hipMemcpyDeviceToDevice, c->stream));
        const int b = L.class_begin[cl], n = L.class_end[cl] - L.class_begin[cl];
        const DevState sc = class_view(c, sw, cl);
        TIMED_LAUNCH(0, launch_edge_kernel(1, c->c128, sc, c->d_items, b, n, c->blocks_per_slice, c->stream));
        TIMED_LAUNCH(1, launch_svd_bwd(c->c128, sc, c->d_items, b, n, c->stream));
        TIMED_LAUNCH(2, launch_edge_kernel(3, c->c128, with_rows(c, sc, b, n), c->d_items, b, n, c->blocks_per_slice,
                                           c->stream));
      }
    }
    for (int cl = C - 1; cl >= 0; --cl) {
      char* sn = c->ws + L.off_snap + (size_t)(cb + cl) * L.state_slot;
      const DevState sp = class_view(c, state_view(c, sn), cb + cl);
      const int b = L.class_begin[cl], n = L.class_end[cl] - L.class_begin[cl];
      double2* ybuf = reinterpret_cast<double2*>(c->ws + L.off_ybuf);
      for (int which = 1; which <= 3; ++which)
        TIMED_LAUNCH(2 + which,
                     launch_adjoint(which, c->c128, with_rows(c, sp, b, n), c->d_items, b, n, c->blocks_per_slice, ybuf,
                                    c->stream));
      TIMED_LAUNCH(8, launch_adjoint(6, c->c128, sp, c->d_items, b, n, c->blocks_per_slice, nullptr, c->stream));
    }
    TIMED_LAUNCH(6, launch_adjoint(5, c->c128, st, c->d_items, 0, (int)L.chunks.size(), c->blocks_per_slice, ck,
                                   c->stream));
  }
  HIP_TRY(c, launch_adjoint(7, c->c128, st, c->d_items, 0, (int)L.chunks.size(), c->blocks_per_slice, nullptr,
                            c->stream));
  std::vector<double> th((size_t)c->n_inst * 2);
  HIP_TRY(c, hipMemcpyAsync(th.data(), st.thbar, th.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  gpeps_status s = check_status_word(c);
  if (s != GPEPS_OK) return s;
  for (int k = 0; k < c->n_inst; ++k) {
    if (dtheta_h) dtheta_h[k] = th[2 * k];
    if (dtheta_j) dtheta_j[k] = th[2 * k + 1];
  }
  return GPEPS_OK;
}

}  // namespace

extern "C" {

gpeps_status gpeps_stats(gpeps_ctx* c, int64_t* out, int32_t n) {
  if (!c || !out || n < 0) return fail(c, GPEPS_ERR_ARG, "ctx and out are required, n >= 0");
  int64_t v[4] = {0, 0, 0, 0};
  HIP_TRY(c, hipMemcpyAsync(v, c->st.stats, sizeof(v), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < n; ++k) out[k] = k < 4 ? v[k] : 0;
  return GPEPS_OK;
}

gpeps_status gpeps_sync(gpeps_ctx* c) {
  if (!c) return fail(nullptr, GPEPS_ERR_ARG, "ctx is NULL");
  return check_status_word(c);
}

gpeps_status gpeps_time_kernels(gpeps_ctx* c, int32_t steps, int32_t n_kinds, double* avg_ms, int64_t* n_launches,
                                const char** kind_names) {
  if (!c) return fail(nullptr, GPEPS_ERR_ARG, "ctx is NULL");
  if (steps < 0 || n_kinds < 0) return fail(c, GPEPS_ERR_ARG, "steps and n_kinds must be >= 0");
  if (c->steps_done + steps > c->max_steps)
    return fail(c, GPEPS_ERR_STATE, "history full: cfg.max_steps steps already recorded (call gpeps_reset)");
  Timer tm;
  tm.on = true;
  gpeps_status s = GPEPS_OK;
  for (int r = 0; r < steps && s == GPEPS_OK; ++r) {
    s = enqueue_step(c, &tm);
    if (s == GPEPS_OK) c->steps_done++;
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  double tot[kKinds] = {0, 0, 0, 0, 0};
  int64_t cnt[kKinds] = {0, 0, 0, 0, 0};
  for (size_t i = 0; i < tm.kind.size(); ++i) {
    float ms = 0.f;
    if (e == hipSuccess && s == GPEPS_OK) e = hipEventElapsedTime(&ms, tm.ev[2 * i], tm.ev[2 * i + 1]);
    tot[tm.kind[i]] += ms;
    cnt[tm.kind[i]] += 1;
  }
  for (hipEvent_t ev : tm.ev) (void)hipEventDestroy(ev);
  if (s != GPEPS_OK) return s;
  if (e != hipSuccess) return fail(c, GPEPS_ERR_HIP, std::string("kernel timing: ") + hipGetErrorString(e));
  for (int k = 0; k < n_kinds; ++k) {
    if (avg_ms) avg_ms[k] = (k < kKinds && cnt[k]) ? tot[k] / (double)cnt[k] : 0.0;
    if (n_launches) n_launches[k] = k < kKinds ? cnt[k] : 0;
    if (kind_names) kind_names[k] = k < kKinds ? kKindNames[k] : "";
  }
  return check_status_word(c);
}

gpeps_status gpeps_time_backward(gpeps_ctx* c, const double* dl_dz, double* dtheta_h, double* dtheta_j,
                                 int32_t n_kinds, double* avg_ms, int64_t* n_launches, const char** kind_names) {
  if (!c || !dl_dz) return fail(c, GPEPS_ERR_ARG, "ctx and dl_dz are required");
  if (n_kinds < 0) return fail(c, GPEPS_ERR_ARG, "n_kinds must be >= 0");
  if (!c->adjoint) return fail(c, GPEPS_ERR_STATE, "context was created with cfg.adjoint = 0");
  if (c->steps_done < 1) return fail(c, GPEPS_ERR_STATE, "no Trotter step recorded: run GPEPS_STEP first");
  HIP_TRY(c, hipMemcpyAsync(c->ws + c->L.off_dldz, dl_dz, (size_t)c->L.NV * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  Timer tm;
  tm.on = true;
  gpeps_status s = reverse_sweep(c, dtheta_h, dtheta_j, &tm);
  hipError_t e = hipStreamSynchronize(c->stream);
  double tot[kAdjKinds] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  int64_t cnt[kAdjKinds] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (size_t i = 0; i < tm.kind.size(); ++i) {
    float ms = 0.f;
    if (e == hipSuccess && s == GPEPS_OK) e = hipEventElapsedTime(&ms, tm.ev[2 * i], tm.ev[2 * i + 1]);
    tot[tm.kind[i]] += ms;
    cnt[tm.kind[i]] += 1;
  }
  for (hipEvent_t ev : tm.ev) (void)hipEventDestroy(ev);
  if (s != GPEPS_OK) return s;
  if (e != hipSuccess) return fail(c, GPEPS_ERR_HIP, std::string("backward timing: ") + hipGetErrorString(e));
  for (int k = 0; k < n_kinds; ++k) {
    if (avg_ms) avg_ms[k] = (k < kAdjKinds && cnt[k]) ? tot[k] / (double)cnt[k] : 0.0;
    if (n_launches) n_launches[k] = k < kAdjKinds ? cnt[k] : 0;
    if (kind_names) kind_names[k] = k < kAdjKinds ? kAdjKindNames[k] : "";
  }
  return GPEPS_OK;
}

}  // extern "C"

namespace {

void drop_step_graph(gpeps_ctx* c) {
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  if (c->step_graph) (void)hipGraphDestroy(c->step_graph);
  if (c->inv_exec) (void)hipGraphExecDestroy(c->inv_exec);
  if (c->inv_graph) (void)hipGraphDestroy(c->inv_graph);
  c->step_exec = nullptr;
  c->step_graph = nullptr;
  c->inv_exec = nullptr;
  c->inv_graph = nullptr;
}

bool valid_tiles(int qr, int rb, int sv) {
  return (qr == 8 || qr == 16) && (rb == 1 || rb == 2 || rb == 4 || rb == 8) && (sv == 64 || sv == 256);
}

// One timed trial: reset, `steps` steps launched one by one, per-kind total milliseconds.
gpeps_status timed_trial(gpeps_ctx* c, int steps, double* tot) {
  gpeps_status s = gpeps_reset(c);
  if (s) return s;
  Timer tm;
  tm.on = true;
  for (int r = 0; r < steps && s == GPEPS_OK; ++r) {
    s = enqueue_step(c, &tm);
    if (s == GPEPS_OK) c->steps_done++;
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  for (int k = 0; k < kKinds; ++k) tot[k] = 0.0;
  for (size_t i = 0; i < tm.kind.size(); ++i) {
    float ms = 0.f;
    if (e == hipSuccess && s == GPEPS_OK) e = hipEventElapsedTime(&ms, tm.ev[2 * i], tm.ev[2 * i + 1]);
    tot[tm.kind[i]] += ms;
  }
  for (hipEvent_t ev : tm.ev) (void)hipEventDestroy(ev);
  if (s != GPEPS_OK) return s;
  if (e != hipSuccess) return fail(c, GPEPS_ERR_HIP, std::string("autotune timing: ") + hipGetErrorString(e));
  return check_status_word(c);
}

}  // namespace

extern "C" {

gpeps_status gpeps_set_tiles(gpeps_ctx* c, const int32_t* tiles) {
  if (!c) return fail(nullptr, GPEPS_ERR_ARG, "ctx is NULL");
  if (!tiles || !valid_tiles(tiles[0], tiles[1], tiles[2]))
    return fail(c, GPEPS_ERR_ARG, "tiles must be {8 or 16, 1, 2, 4 or 8, 64 or 256}");
  if (c->adjoint && c->steps_done > 0)
    return fail(c, GPEPS_ERR_STATE,
                "the reverse sweep recomputes with the forward tiles: call gpeps_reset before gpeps_set_tiles");
  c->st.tune_qr = tiles[0];
  c->st.tune_rb = tiles[1];
  c->st.tune_svd = tiles[2];
  drop_step_graph(c);
  return GPEPS_OK;
}

gpeps_status gpeps_autotune(gpeps_ctx* c, int32_t steps, int32_t* tiles_out) {
  if (!c) return fail(nullptr, GPEPS_ERR_ARG, "ctx is NULL");
  if (steps < 1 || steps > c->max_steps) return fail(c, GPEPS_ERR_ARG, "steps must be in [1, cfg.max_steps]");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  // candidate triples (QR rows per lane, re-absorb tiles per wave, SVD workgroup size); every value
  // of a kernel's own parameter is timed at least once and repeated values are averaged
  const int qr[4] = {16, 8, 16, 8};
  const int rb[4] = {1, 2, 4, 8};
  const int sv[4] = {256, 64, 64, 256};
  const int trials = 4;
  double tot[kKinds];
  c->st.tune_qr = 16;
  c->st.tune_rb = 2;
  c->st.tune_svd = 256;
  drop_step_graph(c);
  gpeps_status s = timed_trial(c, steps, tot);  // warm-up (code objects, caches)
  double t_qr[2] = {0.0, 0.0}, t_rb[4] = {0.0, 0.0, 0.0, 0.0}, t_sv[2] = {0.0, 0.0};
  int n_qr[2] = {0, 0}, n_rb[4] = {0, 0, 0, 0}, n_sv[2] = {0, 0};
  for (int t = 0; t < trials && s == GPEPS_OK; ++t) {
    c->st.tune_qr = qr[t];
    c->st.tune_rb = rb[t];
    c->st.tune_svd = c->D <= 16 ? sv[t] : 256;
    drop_step_graph(c);
    s = timed_trial(c, steps, tot);
    const int iq = qr[t] == 16 ? 0 : 1, is = sv[t] == 256 ? 0 : 1;
    t_qr[iq] += tot[1];
    n_qr[iq]++;
    t_rb[t] += tot[3];
    n_rb[t]++;
    if (c->D <= 16) {
      t_sv[is] += tot[2];
      n_sv[is]++;
    }
  }
  auto avg = [](double t, int n) { return n ? t / n : 1e300; };
  c->st.tune_qr = avg(t_qr[1], n_qr[1]) < avg(t_qr[0], n_qr[0]) ? 8 : 16;
  int best = 0;
  for (int t = 1; t < trials; ++t)
    if (avg(t_rb[t], n_rb[t]) < avg(t_rb[best], n_rb[best])) best = t;
  c->st.tune_rb = rb[best];
  c->st.tune_svd = (c->D <= 16 && avg(t_sv[1], n_sv[1]) < avg(t_sv[0], n_sv[0])) ? 64 : 256;
  if (s != GPEPS_OK) {
    c->st.tune_qr = 16;
    c->st.tune_rb = 2;
    c->st.tune_svd = 256;
  }
  drop_step_graph(c);
  gpeps_status r = gpeps_reset(c);
  if (s != GPEPS_OK) return s;
  if (r != GPEPS_OK) return r;
  if (tiles_out) {
    tiles_out[0] = c->st.tune_qr;
    tiles_out[1] = c->st.tune_rb;
    tiles_out[2] = c->st.tune_svd;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return GPEPS_OK;
}

gpeps_status gpeps_destroy(gpeps_ctx* c) {
  if (!c) return GPEPS_OK;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  if (c->step_graph) (void)hipGraphDestroy(c->step_graph);
  if (c->inv_exec) (void)hipGraphExecDestroy(c->inv_exec);
  if (c->inv_graph) (void)hipGraphDestroy(c->inv_graph);
  delete c;
  if (e != hipSuccess) return fail(nullptr, GPEPS_ERR_HIP, std::string("gpeps_destroy: ") + hipGetErrorString(e));
  return GPEPS_OK;
}

const char* gpeps_last_error(const gpeps_ctx* c) { return c ? c->err.c_str() : g_thread_error.c_str(); }

}  // extern "C"
