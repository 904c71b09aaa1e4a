// Batches of (E, k) instances of uneven size: a native scheduler over the batched kernels.
//
// The paper runs independent energy points side by side (Sec. 4, its outer levels of parallelism).
// On one GPU that becomes: group the instances by block size s (every kernel of a group then shares
// one tile shape), sort each group by block count nb (largest first) and split it into chunks that
// fit the plan's memory.  A chunk runs the whole hot path in lockstep: at recursion step t only the
// instances with more than t blocks are launched, so an uneven chunk does exactly its own work.
// Groups run on their own streams and overlap.  The enqueued work of each group can be captured once
// as a short sequence of bounded graph segments, so an execution is a few graph launches per group.  An
// autotuner times candidate LU panel widths, LU product tiles and chunk sizes per group on the group's
// own smallest instances before capture.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "drivers.hpp"
#include "lu.hpp"

namespace {

using namespace ss;

struct Chunk {
  int first = 0, count = 0;  // positions in the group's sorted order
  RaggedBatch rb;            // device pointers into the group's tables
  // device tables of this chunk
  const ss_c128 **lead_tab = nullptr;
  ss_c128 **psi_tab = nullptr;
  int *orig = nullptr;
  bool any_psi = false;
};

struct Group {
  int s = 0;
  std::vector<int> order;  // caller indices, sorted by nb (largest first)
  ss_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int chunk = 0, lu_width = 0, lu_tile = 0;
  double tune_ms = 0.0;
  std::vector<Chunk> chunks;
  void *tables = nullptr;  // one device allocation holding every chunk's tables
  void *work = nullptr;    // Q, sigma, inj, gc, T, info of one chunk
  ss_c128 *Q = nullptr, *sigma = nullptr, *inj = nullptr, *gc = nullptr;
  double *T = nullptr;
  int *info = nullptr;  // [4][chunk]
  // the group's captured work (when the plan uses graphs): segments replayed in order on its stream
  std::vector<hipGraph_t> graphs;
  std::vector<hipGraphExec_t> execs;
  size_t nodes = 0;
};

__global__ void k_plan_scatter(const double *Tc, const int *ic, const int *orig, int count, int cap, double *T,
                               int *info) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  const int o = orig[j];
  T[2 * o] = Tc[2 * j];
  T[2 * o + 1] = Tc[2 * j + 1];
  for (int k = 0; k < 4; ++k) info[4 * o + k] = ic[k * cap + j];
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// A group's work is captured as a sequence of graphs of at most about kGraphSegmentNodes nodes each
// (ss_plan_opts::graph_segment_nodes), replayed in order on the group's stream.  Instantiating captured
// graphs of about 10^4 to 10^5 kernel nodes (long single dependency chains) ended the host process with
// a segmentation fault in this runtime, while graphs of a few thousand nodes replay correctly; segments
// keep every instantiated graph in that range.  A segment above kMaxGraphNodes (a segment grows by at
// most one launch scope past its limit) makes the plan fall back to a sync-free enqueue.
constexpr size_t kGraphSegmentNodes = 2048;
constexpr size_t kMaxGraphNodes = 8192;

}  // namespace

struct ss_plan {
  ss_ctx *ctx = nullptr;  // caller's context: device and launch stream (not touched by ss_plan_destroy)
  int device = 0;
  int n = 0;
  std::vector<ss_instance> inst;
  ss_plan_opts opts{};
  double *T = nullptr;
  int *info = nullptr;
  std::vector<Group> groups;
  hipEvent_t start = nullptr, finish = nullptr;
  hipStream_t origin = nullptr;  // the stream the batch forks from (captured when a graph is built)
  bool graphs = false;           // every group replays its own captured graph segments
  size_t graph_nodes = 0;       // summed over the groups
  size_t graph_segments = 0;    // summed over the groups
  long long graph_refused = 0;  // nodes of a capture with a segment judged too large to instantiate
};

namespace {

// device bytes one instance of the group holds while its chunk runs (upper bound): recursion slots of
// both systems and Q (4 nb s^2), decimation state and sigma (14 s^2), recursion and corner systems,
// corner work and G corner (24 s^2), and the m-column blocks of the corner solve and the injection
size_t instance_bytes(int s, int nb, int m) {
  const size_t e = sizeof(ss_c128), ss2 = (size_t)s * s;
  return e * ((4 * (size_t)nb + 38) * ss2 + 6 * (size_t)s * m) + 4096;
}

ss_status build_chunks(ss_plan *p, Group &g, int chunk) {
  g.chunks.clear();
  const int cnt = (int)g.order.size();
  for (int f = 0; f < cnt; f += chunk) {
    Chunk c;
    c.first = f;
    c.count = std::min(chunk, cnt - f);
    g.chunks.push_back(c);
  }
  // one table allocation: per chunk tab[4c], lead[4c], psi[c] pointers, nbv[c], orig[c], boff[c],
  // xoff[2c], E[c]
  std::vector<size_t> offs;
  size_t total = 0;
  for (auto &c : g.chunks) {
    offs.push_back(total);
    total += align256(sizeof(void *) * 9 * c.count) + align256(sizeof(int) * 2 * c.count) +
             align256(sizeof(long) * 3 * c.count) + align256(sizeof(double) * c.count);
  }
  if (g.tables) (void)hipFree(g.tables);
  g.tables = nullptr;
  if (hipMalloc(&g.tables, std::max<size_t>(total, 256)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(p->ctx, SS_ERR_NOMEM, "ss_plan_create: table allocation failed");
  }
  std::vector<char> host(std::max<size_t>(total, 256));
  size_t qmax = 0;
  for (size_t ci = 0; ci < g.chunks.size(); ++ci) {
    Chunk &c = g.chunks[ci];
    char *hb = host.data() + offs[ci];
    char *db = (char *)g.tables + offs[ci];
    const int C = c.count;
    const void **tab = (const void **)hb;                 // 4C data, 4C lead, C psi
    int *nbv = (int *)(hb + align256(sizeof(void *) * 9 * C));
    int *orig = nbv + C;
    long *boff = (long *)(hb + align256(sizeof(void *) * 9 * C) + align256(sizeof(int) * 2 * C));
    long *xoff = boff + C;
    double *E = (double *)((char *)boff + align256(sizeof(long) * 3 * C));
    const size_t o_nbv = (char *)nbv - hb, o_orig = (char *)orig - hb, o_boff = (char *)boff - hb,
                 o_xoff = (char *)xoff - hb, o_E = (char *)E - hb;
    long blocks = 0;
    c.any_psi = false;
    c.rb.act.assign(p->inst[g.order[c.first]].nb, 0);
    const long ss2 = (long)g.s * g.s;
    for (int j = 0; j < C; ++j) {
      const ss_instance &in = p->inst[g.order[c.first + j]];
      tab[4 * j + 0] = in.H_diag;
      tab[4 * j + 1] = in.H_upper;
      tab[4 * j + 2] = in.S_diag;
      tab[4 * j + 3] = in.S_upper;
      tab[4 * C + 4 * j + 0] = in.H00;
      tab[4 * C + 4 * j + 1] = in.H01;
      tab[4 * C + 4 * j + 2] = in.S00;
      tab[4 * C + 4 * j + 3] = in.S01;
      tab[8 * C + j] = in.psi;
      c.any_psi = c.any_psi || in.psi != nullptr;
      nbv[j] = in.nb;
      orig[j] = g.order[c.first + j];
      boff[j] = blocks;
      xoff[2 * j] = 2 * blocks * ss2;
      xoff[2 * j + 1] = (2 * blocks + in.nb) * ss2;
      E[j] = in.E;
      for (int t = 0; t < in.nb; ++t) c.rb.act[t] = j + 1;
      blocks += in.nb;
    }
    c.rb.s = g.s;
    c.rb.batch = C;
    c.rb.nb_max = p->inst[g.order[c.first]].nb;
    c.rb.total_blocks = blocks;
    c.rb.tab = (const ss_c128 *const *)db;
    c.lead_tab = (const ss_c128 **)(db + sizeof(void *) * 4 * C);
    c.psi_tab = c.any_psi ? (ss_c128 **)(db + sizeof(void *) * 8 * C) : nullptr;
    c.rb.nbv = (const int *)(db + o_nbv);
    c.orig = (int *)(db + o_orig);
    c.rb.boff = (const long *)(db + o_boff);
    c.rb.xoff = (const long *)(db + o_xoff);
    c.rb.E = (const double *)(db + o_E);
    qmax = std::max(qmax, (size_t)blocks);
  }
  if (hipMemcpy(g.tables, host.data(), total, hipMemcpyHostToDevice) != hipSuccess)
    return fail(p->ctx, SS_ERR_DEVICE, "ss_plan_create: table upload failed");
  // per-chunk outputs
  const size_t ss2 = (size_t)g.s * g.s;
  const int m = p->opts.m;
  const size_t bQ = align256(sizeof(ss_c128) * qmax * 2 * ss2), bS = align256(sizeof(ss_c128) * chunk * 2 * ss2),
               bI = align256(sizeof(ss_c128) * chunk * 2 * (size_t)g.s * std::max(m, 1)),
               bG = align256(sizeof(ss_c128) * chunk * 4 * ss2), bT = align256(sizeof(double) * 2 * chunk),
               bN = align256(sizeof(int) * 4 * chunk);
  if (g.work) (void)hipFree(g.work);
  g.work = nullptr;
  if (hipMalloc(&g.work, bQ + bS + bI + bG + bT + bN) != hipSuccess) {
    (void)hipGetLastError();
    return fail(p->ctx, SS_ERR_NOMEM, "ss_plan_create: chunk buffer allocation failed");
  }
  char *w = (char *)g.work;
  g.Q = (ss_c128 *)w;
  g.sigma = (ss_c128 *)(w += bQ);
  g.inj = (ss_c128 *)(w += bS);
  g.gc = (ss_c128 *)(w += bI);
  g.T = (double *)(w += bG);
  g.info = (int *)(w += bT);
  g.chunk = chunk;
  return SS_OK;
}

// Enqueue one chunk of a group on the group's stream.
ss_status run_chunk(ss_plan *p, Group &g, const Chunk &c) {
  ss_ctx *x = g.ctx;
  const int C = c.count, s = g.s, m = p->opts.m;
  int *i_sig = g.info, *i_pre = g.info + g.chunk, *i_obc = g.info + 2 * g.chunk, *i_it = g.info + 3 * g.chunk;
  SS_TRY(lead_selfenergy(x, C, s, C, nullptr, nullptr, nullptr, nullptr, nullptr, c.rb.E, p->opts.eta,
                         p->opts.sigma_tol, p->opts.sigma_passes, g.sigma, i_it, nullptr, i_sig, c.lead_tab));
  SS_TRY(precompute_ragged(x, c.rb, p->opts.absorb, SS_PREC_FP64, g.Q, i_pre));
  const int mm = c.any_psi ? m : 0;
  if (mm > 0) SS_TRY(injection_left(x, C, s, g.sigma, 0.0, mm, g.inj, nullptr));
  SS_TRY(apply_obc_ragged(x, c.rb, g.Q, g.sigma, p->opts.absorb, mm, g.inj, mm > 0 ? c.psi_tab : nullptr, g.gc, i_obc));
  SS_TRY(transmission(x, C, s, g.gc, g.sigma, g.T));
  hipLaunchKernelGGL(k_plan_scatter, dim3(cdiv(C, 256)), dim3(256), 0, x->stream, (const double *)g.T,
                     (const int *)g.info, (const int *)c.orig, C, g.chunk, p->T, p->info);
  return check_launch(x, "ss_plan: scatter");
}

// Enqueue a group's chunks; on failure `msg` names the group and the error (p->ctx is not touched, so
// groups may enqueue from different host threads).
ss_status enqueue_group(ss_plan *p, Group &g, std::string &msg) {
  for (const Chunk &c : g.chunks) {
    ss_status st = run_chunk(p, g, c);
    if (st != SS_OK) {
      msg = "group s=" + std::to_string(g.s) + ": " + g.ctx->err;
      return st;
    }
  }
  return SS_OK;
}

ss_status run_group(ss_plan *p, Group &g) {
  std::string msg;
  const ss_status st = enqueue_group(p, g, msg);
  return st == SS_OK ? SS_OK : fail(p->ctx, st, msg);
}

// Launch a group's captured graph segments in order on its stream.
ss_status launch_group(Group &g, std::string &msg) {
  for (hipGraphExec_t e : g.execs)
    if (hipGraphLaunch(e, g.stream) != hipSuccess) {
      msg = "group s=" + std::to_string(g.s) + ": graph launch failed";
      return SS_ERR_DEVICE;
    }
  return SS_OK;
}

// Enqueue the whole batch on `origin`: every group forks from it and joins back into it.  Each group
// enqueues from a host thread of its own, its captured graph segments (with graphs) or its launches: a
// launch blocks the enqueuing thread while the stream's hardware queue is full, so one thread
// enqueuing group after group would keep every group but the current one idle (the groups would run
// one after the other).
ss_status enqueue(ss_plan *p, hipStream_t origin) {
  if (hipEventRecord(p->start, origin) != hipSuccess) return fail(p->ctx, SS_ERR_DEVICE, "ss_plan: event record failed");
  for (Group &g : p->groups)
    if (hipStreamWaitEvent(g.stream, p->start, 0) != hipSuccess)
      return fail(p->ctx, SS_ERR_DEVICE, "ss_plan: stream wait failed");
  if (p->groups.size() == 1) {
    std::string msg;
    const ss_status st = p->graphs ? launch_group(p->groups[0], msg) : enqueue_group(p, p->groups[0], msg);
    if (st != SS_OK) return fail(p->ctx, st, msg);
  } else {
    const size_t ng = p->groups.size();
    std::vector<ss_status> st(ng, SS_OK);
    std::vector<std::string> msg(ng);
    std::vector<std::thread> th;
    th.reserve(ng);
    for (size_t i = 0; i < ng; ++i)
      th.emplace_back([p, i, &st, &msg] {
        if (hipSetDevice(p->device) != hipSuccess) {
          st[i] = SS_ERR_DEVICE;
          msg[i] = "hipSetDevice failed in an enqueue thread";
          return;
        }
        st[i] = p->graphs ? launch_group(p->groups[i], msg[i]) : enqueue_group(p, p->groups[i], msg[i]);
      });
    for (std::thread &t : th) t.join();
    for (size_t i = 0; i < ng; ++i)
      if (st[i] != SS_OK) return fail(p->ctx, st[i], msg[i]);
  }
  for (Group &g : p->groups)
    if (hipEventRecord(g.done, g.stream) != hipSuccess || hipStreamWaitEvent(origin, g.done, 0) != hipSuccess)
      return fail(p->ctx, SS_ERR_DEVICE, "ss_plan: join failed");
  return SS_OK;
}

// Capture every group's work (capture on the group's stream) into graph segments of about
// graph_segment_nodes nodes each: the group's context closes the current capture at a launch site once
// it holds that many nodes and opens the next.  A segment above kMaxGraphNodes makes the plan fall back
// to the sync-free enqueue for all groups.
ss_status capture_groups(ss_plan *p) {
  size_t total = 0, nseg = 0;
  bool too_big = false;
  const size_t limit = p->opts.graph_segment_nodes > 0 ? (size_t)p->opts.graph_segment_nodes : kGraphSegmentNodes;
  auto drop = [&]() {
    for (Group &g : p->groups) {
      for (hipGraph_t gr : g.graphs) (void)hipGraphDestroy(gr);
      g.graphs.clear();
      g.nodes = 0;
    }
  };
  for (Group &g : p->groups) {
    if (hipStreamBeginCapture(g.stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      drop();
      return fail(p->ctx, SS_ERR_DEVICE, "ss_plan_create: stream capture could not start");
    }
    g.ctx->seg_graphs = &g.graphs;
    g.ctx->seg_limit = limit;
    g.ctx->seg_failed = false;
    const ss_status st = run_group(p, g);
    g.ctx->seg_graphs = nullptr;
    hipGraph_t last = nullptr;
    const hipError_t ec = hipStreamEndCapture(g.stream, &last);
    if (last) g.graphs.push_back(last);
    if (st != SS_OK) {
      drop();
      return st;
    }
    if (g.ctx->seg_failed || ec != hipSuccess || !last) {
      drop();
      return fail(p->ctx, SS_ERR_DEVICE, "ss_plan_create: capture failed");
    }
    for (hipGraph_t gr : g.graphs) {
      size_t n = 0;
      if (hipGraphGetNodes(gr, nullptr, &n) != hipSuccess) {
        drop();
        return fail(p->ctx, SS_ERR_DEVICE, "ss_plan_create: graph node count failed");
      }
      g.nodes += n;
      if (n > kMaxGraphNodes) too_big = true;
    }
    total += g.nodes;
    nseg += g.graphs.size();
  }
  if (too_big) {
    p->graph_refused = (long long)total;
    drop();
    return SS_OK;
  }
  for (Group &g : p->groups)
    for (hipGraph_t gr : g.graphs) {
      hipGraphExec_t e = nullptr;
      if (hipGraphInstantiate(&e, gr, nullptr, nullptr, 0) != hipSuccess || !e)
        return fail(p->ctx, SS_ERR_DEVICE, "ss_plan_create: graph instantiation failed");
      g.execs.push_back(e);
    }
  p->graphs = true;
  p->graph_nodes = total;
  p->graph_segments = nseg;
  return SS_OK;
}

// Time candidate (panel width, product tile, chunk size) triples on the group's smallest instances and
// keep the one with the least time per recursion block.
ss_status autotune(ss_plan *p, Group &g, int chunk_max) {
  std::vector<int> widths;
  for (int w : {32, 16, 8})
    if (lu_panel_width_ok(g.s, w)) widths.push_back(w);
  std::vector<int> chunks = {chunk_max};
  if (chunk_max >= 4) chunks.push_back((chunk_max + 1) / 2);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(p->ctx, SS_ERR_DEVICE, "ss_plan: event creation failed");
  double best = 1e300;
  int best_w = widths[0], best_c = chunk_max, best_t = 0;
  std::vector<int> full = g.order;
  ss_status st = SS_OK;
  for (int c : chunks) {
    // probe batch: the c instances with the fewest blocks
    const int take = std::min<int>(c, (int)full.size());
    g.order.assign(full.end() - take, full.end());
    st = build_chunks(p, g, take);
    if (st != SS_OK) break;
    long blocks = 0;
    for (int idx : g.order) blocks += p->inst[idx].nb;
    for (int w : widths) {
      for (int tile : {0, 1}) {
        g.ctx->lu_width = w;
        g.ctx->lu_tile = tile;
        // once untimed (workspaces grow, code loads), then timed
        st = run_group(p, g);
        if (st == SS_OK && hipEventRecord(e0, g.stream) == hipSuccess && (st = run_group(p, g)) == SS_OK &&
            hipEventRecord(e1, g.stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess) {
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          const double per = ms / std::max<long>(blocks, 1);
          if (per < best) { best = per; best_w = w; best_c = c; best_t = tile; g.tune_ms = ms; }
        }
        if (st != SS_OK) break;
      }
      if (st != SS_OK) break;
    }
    if (st != SS_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g.order = full;
  if (st != SS_OK) return fail(p->ctx, st, "ss_plan: a tuning candidate failed: " + g.ctx->err);
  g.ctx->lu_width = best_w;
  g.lu_width = best_w;
  g.ctx->lu_tile = best_t;
  g.lu_tile = best_t;
  if (hipStreamSynchronize(g.stream) != hipSuccess) return fail(p->ctx, SS_ERR_DEVICE, "ss_plan: tuning failed");
  return build_chunks(p, g, best_c);
}

void release(ss_plan *p) {
  if (p->origin) (void)hipStreamSynchronize(p->origin);
  for (Group &g : p->groups) {
    if (g.stream) (void)hipStreamSynchronize(g.stream);
    for (hipGraphExec_t e : g.execs) (void)hipGraphExecDestroy(e);
    for (hipGraph_t gr : g.graphs) (void)hipGraphDestroy(gr);
    if (g.ctx) ss_destroy(g.ctx);
    if (g.tables) (void)hipFree(g.tables);
    if (g.work) (void)hipFree(g.work);
    if (g.done) (void)hipEventDestroy(g.done);
    if (g.stream) (void)hipStreamDestroy(g.stream);
  }
  if (p->start) (void)hipEventDestroy(p->start);
  if (p->finish) (void)hipEventDestroy(p->finish);
  if (p->origin) (void)hipStreamDestroy(p->origin);
  delete p;
}

}  // namespace

extern "C" {

ss_status ss_plan_create(ss_ctx *ctx, int n, const ss_instance *inst, const ss_plan_opts *opts, double *T,
                         int *info, ss_plan **out) {
  if (!ctx || !out) return SS_ERR_ARG;
  *out = nullptr;
  ctx->err.clear();
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SS_ERR_DEVICE, "hipSetDevice failed");
  if (n < 1 || !inst || !opts || !T || !info) return fail(ctx, SS_ERR_ARG, "ss_plan_create: null argument or n < 1");
  if (opts->m < 0 || opts->m > SS_MAX_S || opts->eta < 0 || !(opts->absorb >= 0) || !std::isfinite(opts->absorb) ||
      opts->sigma_tol < 0 || opts->sigma_passes < 0 || opts->graph_segment_nodes < 0 ||
      opts->graph_segment_nodes > (int)kGraphSegmentNodes * 2)
    return fail(ctx, SS_ERR_ARG, "ss_plan_create: option out of range");
  for (int i = 0; i < n; ++i) {
    const ss_instance &in = inst[i];
    if (in.nb < 1 || in.s < 1) return fail(ctx, SS_ERR_ARG, "ss_plan_create: instance " + std::to_string(i) + " size");
    if (in.s > SS_MAX_S) return fail(ctx, SS_ERR_UNSUPPORTED, "ss_plan_create: s > SS_MAX_S");
    if (!in.H_diag || !in.S_diag || (in.nb > 1 && (!in.H_upper || !in.S_upper)) || !in.H00 || !in.H01 || !in.S00 ||
        !in.S01)
      return fail(ctx, SS_ERR_ARG, "ss_plan_create: instance " + std::to_string(i) + " has a null block pointer");
    if (in.psi && opts->m < 1) return fail(ctx, SS_ERR_ARG, "ss_plan_create: psi requested with m = 0");
  }
  ss_plan *p = new (std::nothrow) ss_plan();
  if (!p) return fail(ctx, SS_ERR_NOMEM, "ss_plan_create: out of host memory");
  p->ctx = ctx;
  p->device = ctx->device;
  p->n = n;
  p->inst.assign(inst, inst + n);
  p->opts = *opts;
  if (p->opts.sigma_passes == 0) {
    // a decimation pass doubles the cell range and the broadening damps a propagating mode over about
    // 1/eta cells, so about log2(1/eta) passes converge; a margin covers slow modes
    const double eta = p->opts.eta > 0 ? p->opts.eta : 1e-60;
    p->opts.sigma_passes = std::min(200, std::max(16, (int)std::ceil(std::log2(1.0 / eta)) + 12));
  }
  if (p->opts.mem_bytes == 0) p->opts.mem_bytes = (size_t)32 << 30;
  p->T = T;
  p->info = info;
  auto bail = [&](ss_status st) {
    const std::string msg = ctx->err;
    release(p);
    ctx->err = msg;
    return st;
  };
  if (hipEventCreateWithFlags(&p->start, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->finish, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&p->origin, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(ctx, SS_ERR_DEVICE, "ss_plan_create: event or stream creation failed"));
  std::map<int, std::vector<int>> by_s;
  for (int i = 0; i < n; ++i) by_s[inst[i].s].push_back(i);
  size_t work_total = 0;
  for (auto &kv : by_s)
    for (int i : kv.second) work_total += (size_t)inst[i].nb * kv.first * kv.first * kv.first / 64 + 1;
  for (auto &kv : by_s) {
    Group g;
    g.s = kv.first;
    g.order = kv.second;
    std::stable_sort(g.order.begin(), g.order.end(), [&](int a, int b) { return inst[a].nb > inst[b].nb; });
    p->groups.push_back(g);
  }
  // memory budget per group: a floor that lets a small group run whole (or at least half of an even
  // split of the budget), and the rest of the budget in proportion to the group's work (nb s^3)
  const int ngroups = (int)p->groups.size();
  std::vector<size_t> floor_b(ngroups), gbytes(ngroups, 0), gwork(ngroups, 0);
  size_t floors = 0;
  for (int gi = 0; gi < ngroups; ++gi) {
    const Group &g = p->groups[gi];
    for (int i : g.order) {
      gbytes[gi] += instance_bytes(g.s, inst[i].nb, p->opts.m);
      gwork[gi] += (size_t)inst[i].nb * g.s * g.s * g.s / 64 + 1;
    }
    floor_b[gi] = std::min(gbytes[gi], p->opts.mem_bytes / (2 * (size_t)ngroups));
    floors += floor_b[gi];
  }
  const size_t rest = p->opts.mem_bytes > floors ? p->opts.mem_bytes - floors : 0;
  int gi = 0;
  for (Group &g : p->groups) {
    const size_t share = floor_b[gi] + (size_t)((double)rest * gwork[gi] / work_total);
    ++gi;
    if (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g.done, hipEventDisableTiming) != hipSuccess)
      return bail(fail(ctx, SS_ERR_DEVICE, "ss_plan_create: stream creation failed"));
    if (ss_create(&g.ctx, ctx->device, g.stream) != SS_OK)
      return bail(fail(ctx, SS_ERR_NOMEM, "ss_plan_create: group context"));
    // the chunk must hold at least the group's largest instance
    int chunk = 0;
    size_t used = 0;
    for (int i : g.order) {
      used += instance_bytes(g.s, inst[i].nb, p->opts.m);
      if (used > share && chunk > 0) break;
      ++chunk;
    }
    ss_status st = p->opts.autotune ? autotune(p, g, chunk) : build_chunks(p, g, chunk);
    if (st != SS_OK) return bail(st);
    if (!p->opts.autotune) g.lu_width = lu_panel_width(g.s);
  }
  // eager pass: grows every workspace to its final size and checks the launches
  ss_status st = enqueue(p, p->origin);
  if (st != SS_OK) return bail(st);
  if (hipStreamSynchronize(p->origin) != hipSuccess)
    return bail(fail(ctx, SS_ERR_DEVICE, "ss_plan_create: first pass failed"));
  for (Group &g : p->groups) g.ctx->sync_free = true;
  if (p->opts.use_graph) {
    st = capture_groups(p);
    if (st != SS_OK) return bail(st);
  }
  *out = p;
  return SS_OK;
}

ss_status ss_plan_execute(ss_plan *p) {
  if (!p) return SS_ERR_ARG;
  ss_ctx *ctx = p->ctx;
  ctx->err.clear();
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SS_ERR_DEVICE, "hipSetDevice failed");
  // ordered after the work already on the caller's stream, and the caller's stream after the batch
  if (hipEventRecord(p->finish, ctx->stream) != hipSuccess || hipStreamWaitEvent(p->origin, p->finish, 0) != hipSuccess)
    return fail(ctx, SS_ERR_DEVICE, "ss_plan_execute: stream ordering failed");
  SS_TRY(enqueue(p, p->origin));
  if (hipEventRecord(p->finish, p->origin) != hipSuccess || hipStreamWaitEvent(ctx->stream, p->finish, 0) != hipSuccess)
    return fail(ctx, SS_ERR_DEVICE, "ss_plan_execute: stream ordering failed");
  return SS_OK;
}

ss_status ss_plan_describe(const ss_plan *p, int group, int *s, int *count, int *chunk, int *lu_width,
                           double *tune_ms) {
  if (!p || group < 0 || group >= (int)p->groups.size()) return SS_ERR_ARG;
  const Group &g = p->groups[group];
  if (s) *s = g.s;
  if (count) *count = (int)g.order.size();
  if (chunk) *chunk = g.chunk;
  if (lu_width) *lu_width = g.lu_width;
  if (tune_ms) *tune_ms = g.tune_ms;
  return SS_OK;
}

int ss_plan_groups(const ss_plan *p) { return p ? (int)p->groups.size() : 0; }

int ss_plan_lu_tile(const ss_plan *p, int group) {
  if (!p || group < 0 || group >= (int)p->groups.size()) return -1;
  return p->groups[group].lu_tile;
}

long long ss_plan_graph_nodes(const ss_plan *p) {
  if (!p) return 0;
  return p->graph_nodes ? (long long)p->graph_nodes : -p->graph_refused;
}

int ss_plan_graph_segments(const ss_plan *p) { return p ? (int)p->graph_segments : 0; }

void ss_plan_destroy(ss_plan *p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  release(p);  // waits for the plan's own streams
}

}  // extern "C"
