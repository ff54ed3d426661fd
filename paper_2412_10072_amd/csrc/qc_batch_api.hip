// Host side of the batched solve: validation of every problem, work-item
// construction and bucketing, the hipGraph of the bucket launches, and the
// autotuner that picks (waves per workgroup, rows per step) per bucket by
// timing the candidates on the batch itself.

#include <numeric>

#include "qc_batch.h"
#include "qc_host.h"
#include "qc_hostcheck.h"

using namespace qc;

namespace {

// Buckets: channel-width class (<= 16, <= 32, wider) x size class.
constexpr int N_WIDTH = 3;
constexpr int N_SIZE = 2;
constexpr int N_BUCKET = N_WIDTH * N_SIZE;
constexpr long long SMALL_SAMPLES = 1 << 16;

int width_class(int n_ch) { return n_ch <= 16 ? 0 : (n_ch <= 32 ? 1 : 2); }

struct Bucket {
  int begin = 0, count = 0;
  int waves = 4, rps = 1;
  int grid = 0;
  size_t lds = 0;
  float ms = -1.f;     // tuned time (ms), negative if untuned
};

}  // namespace

struct qc_batch {
  qc_ctx* ctx = nullptr;
  int n_prob = 0, n_items = 0;
  int prec_mixed = 0, vis_c128 = 0, max_ant = 1;
  int lm = 0;                             // Levenberg-Marquardt damping for every problem
  int n_int = 0;                          // intervals over every problem
  int all_diag = 1;                       // every problem's term is DIAGONAL
  int warm = 0;                           // some problem has a warm-start fallback reference
  double tol = 1e-6;
  int max_iter = 100;
  std::vector<BatchProb> probs;
  std::vector<qc_problem> problems;       // the caller's problems (device pointers)
  BatchProb* d_probs = nullptr;
  BatchItem* d_items = nullptr;
  int* d_queue = nullptr;                 // [N_BUCKET]
  Bucket bucket[N_BUCKET];
  hipStream_t cs = nullptr;               // capture stream
  hipStream_t bs[N_BUCKET] = {};
  hipEvent_t fork = nullptr, join[N_BUCKET] = {};
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int n_cu = 256;
};

namespace {

qc_status bucket_config(qc_batch* b, Bucket& k, int waves, int rps) {
  qc_ctx* ctx = b->ctx;
  k.waves = waves;
  k.rps = rps;
  k.lds = batch_lds_bytes(b->prec_mixed, b->max_ant, waves);
  if (k.lds > 160 * 1024) return fail(ctx, QC_E_UNSUPPORTED, "batch needs %zu B of LDS", k.lds);
  void* kern = batch_kernel_ptr(b->prec_mixed, b->vis_c128, rps, b->lm, b->warm);
  if (k.lds > 64 * 1024)
    HIP_TRY(ctx, hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)k.lds));
  int per_cu = 0;
  HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * waves, k.lds));
  per_cu = std::max(per_cu, 1);
  k.grid = std::max(1, std::min(k.count, b->n_cu * per_cu));
  return QC_OK;
}

BatchArgs bucket_args(qc_batch* b, int i) {
  BatchArgs a;
  a.probs = b->d_probs;
  a.items = b->d_items;
  a.item_begin = b->bucket[i].begin;
  a.n_items = b->bucket[i].count;
  a.queue = b->d_queue + i;
  a.tol = b->tol;
  a.max_iter = b->max_iter;
  a.err = b->ctx->d_err;
  return a;
}

qc_status launch_bucket(qc_batch* b, int i, hipStream_t s) {
  const Bucket& k = b->bucket[i];
  if (k.count == 0) return QC_OK;
  BatchArgs a = bucket_args(b, i);
  HIP_TRY(b->ctx, launch_batch_bucket(a, batch_kernel_ptr(b->prec_mixed, b->vis_c128, k.rps, b->lm, b->warm), k.waves, k.lds,
                                      k.grid, s));
  return QC_OK;
}

void drop_graph(qc_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// One graph: zero the queue counters, then every non-empty bucket on its own
// branch, joined back into the capture stream.
qc_status build_graph(qc_batch* b) {
  qc_ctx* ctx = b->ctx;
  drop_graph(b);
  HIP_TRY(ctx, hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal));
  qc_status st = QC_OK;
  hipError_t e = launch_zero_ints(b->d_queue, N_BUCKET, b->cs);
  if (e == hipSuccess) e = hipEventRecord(b->fork, b->cs);
  for (int i = 0; i < N_BUCKET && e == hipSuccess; ++i) {
    if (b->bucket[i].count == 0) continue;
    e = hipStreamWaitEvent(b->bs[i], b->fork, 0);
    if (e == hipSuccess) {
      st = launch_bucket(b, i, b->bs[i]);
      if (st != QC_OK) break;
    }
    if (e == hipSuccess) e = hipEventRecord(b->join[i], b->bs[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->cs, b->join[i], 0);
  }
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->cs, &g);
  if (st != QC_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return fail(ctx, QC_E_DEVICE, "batch graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  b->graph = g;
  HIP_TRY(ctx, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return QC_OK;
}

}  // namespace

extern "C" {

qc_status qc_batch_create(qc_ctx* ctx, const qc_problem* problems, int32_t n_problem, const qc_solve_opts* opts,
                          qc_batch** out) {
  if (!ctx) return QC_E_ARG;
  if (!out) return fail(ctx, QC_E_ARG, "out is NULL");
  *out = nullptr;
  if (!problems || n_problem <= 0) return fail(ctx, QC_E_ARG, "no problems");
  if (!opts) return fail(ctx, QC_E_ARG, "opts is NULL");
  const int prec_v = enum_value(opts->prec), damp_v = enum_value(opts->damping);
  if (prec_v != QC_PREC_FP64 && prec_v != QC_PREC_MIXED) return fail(ctx, QC_E_ARG, "bad precision %d", prec_v);
  if (damp_v < QC_DAMP_FULL || damp_v > QC_DAMP_LM) return fail(ctx, QC_E_ARG, "bad damping %d", damp_v);
  if (opts->max_iter < 0) return fail(ctx, QC_E_ARG, "max_iter < 0");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(opts->stream);
  qc_batch* b = new qc_batch();
  b->ctx = ctx;
  b->n_prob = n_problem;
  b->prec_mixed = opts->prec == QC_PREC_MIXED;
  b->lm = opts->damping == QC_DAMP_LM;
  b->vis_c128 = enum_value(problems[0].vis.dtype) == QC_C128;
  b->tol = opts->tol;
  b->max_iter = opts->max_iter;
  b->problems.assign(problems, problems + n_problem);
  std::vector<BatchItem> items;
  std::vector<long long> cost;
  auto bail = [&](qc_status st) {
    qc_batch_destroy(b);
    return st;
  };
  for (int i = 0; i < n_problem; ++i) {
    const qc_problem& P = problems[i];
    if ((enum_value(P.vis.dtype) == QC_C128) != (b->vis_c128 != 0))
      return bail(fail(ctx, QC_E_ARG, "problem %d: every problem must have the same data dtype", i));
    if (b->prec_mixed && enum_value(P.vis.dtype) != QC_C64)
      return bail(fail(ctx, QC_E_ARG, "MIXED precision needs complex64 data"));
    if (enum_value(P.term.type) != QC_TERM_DIAGONAL && enum_value(P.term.type) != QC_TERM_COMPLEX2X2)
      return bail(fail(ctx, QC_E_UNSUPPORTED, "problem %d: batched terms must be DIAGONAL or COMPLEX2X2", i));
    if (P.vis.n_dir != 1 || P.term.n_gdir != 1)
      return bail(fail(ctx, QC_E_UNSUPPORTED, "problem %d: batched problems have one direction", i));
    std::vector<HostMaps> maps;
    qc_status st = prepare(ctx, &P.vis, &P.term, 1, 0, maps, s);
    if (st != QC_OK) {
      ctx->msg = "problem " + std::to_string(i) + ": " + ctx->msg;
      return bail(st);
    }
    std::vector<long long> rlo(P.term.n_gt), rhi(P.term.n_gt);
    HIP_TRY(ctx, hipMemcpyAsync(rlo.data(), ctx->d_rowlo, sizeof(long long) * rlo.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(rhi.data(), ctx->d_rowhi, sizeof(long long) * rhi.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    BatchProb bp;
    memset(&bp, 0, sizeof bp);
    ChainArgs ca;
    fill_args(&P.vis, &P.term, 1, 0, bp.vis, ca);
    bp.term = ca.t[0];
    bp.gains = reinterpret_cast<double2*>(P.term.gains);
    bp.gflags = P.term.gain_flags;
    bp.iters = P.stats.iters;
    bp.converged = P.stats.converged;
    bp.chisq_first = P.stats.chisq_first;
    bp.chisq_last = P.stats.chisq_last;
    bp.chisq_ref = P.chisq_ref;
    if (P.chisq_ref) b->warm = 1;
    bp.restarted = P.stats.restarted;
    bp.damping = resolve_damping(opts->damping, P.term);
    bp.int_base = b->n_int;
    b->n_int += P.term.n_gt * P.term.n_gf;
    if (P.term.type != QC_TERM_DIAGONAL) b->all_diag = 0;
    b->probs.push_back(bp);
    b->max_ant = std::max(b->max_ant, P.vis.n_ant);
    for (int gt = 0; gt < P.term.n_gt; ++gt)
      for (int gf = 0; gf < P.term.n_gf; ++gf) {
        BatchItem it;
        it.r_lo = rlo[gt];
        it.r_hi = rhi[gt];
        it.c_lo = ctx->h_clo[gf];
        it.c_hi = ctx->h_chi[gf];
        it.prob = i;
        it.gt = gt;
        it.gf = gf;
        it.pad = 0;
        items.push_back(it);
      }
  }
  // bucket, then largest first inside a bucket
  std::vector<int> key(items.size());
  std::vector<long long> size(items.size());
  for (size_t k = 0; k < items.size(); ++k) {
    const BatchItem& it = items[k];
    const long long smp = (it.r_hi - it.r_lo) * (long long)(it.c_hi - it.c_lo);
    size[k] = smp * (b->probs[it.prob].term.kind == KIND_C2X2 ? 2 : 1);
    key[k] = width_class(it.c_hi - it.c_lo) * N_SIZE + (smp < SMALL_SAMPLES ? 0 : 1);
  }
  std::vector<size_t> order(items.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
    return key[x] != key[y] ? key[x] < key[y] : size[x] > size[y];
  });
  std::vector<BatchItem> sorted(items.size());
  for (size_t k = 0; k < order.size(); ++k) sorted[k] = items[order[k]];
  for (size_t k = 0; k < order.size(); ++k) {
    Bucket& bk = b->bucket[key[order[k]]];
    if (bk.count == 0) bk.begin = (int)k;
    bk.count++;
  }
  b->n_items = (int)sorted.size();
  int dev_cu = 0;
  HIP_TRY(ctx, hipDeviceGetAttribute(&dev_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  b->n_cu = std::max(dev_cu, 1);
  for (int i = 0; i < N_BUCKET; ++i) {
    const int w = i / N_SIZE, z = i % N_SIZE;
    qc_status st = bucket_config(b, b->bucket[i], z == 0 ? 2 : 4, w == 0 ? 4 : (w == 1 ? 2 : 1));
    if (st != QC_OK) return bail(st);
  }
  if (hipMalloc(reinterpret_cast<void**>(&b->d_probs), sizeof(BatchProb) * b->probs.size()) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&b->d_items), sizeof(BatchItem) * std::max<size_t>(sorted.size(), 1)) !=
          hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&b->d_queue), sizeof(int) * N_BUCKET) != hipSuccess)
    return bail(fail(ctx, QC_E_NOMEM, "batch descriptors"));
  HIP_TRY(ctx, hipMemcpy(b->d_probs, b->probs.data(), sizeof(BatchProb) * b->probs.size(), hipMemcpyHostToDevice));
  if (!sorted.empty())
    HIP_TRY(ctx, hipMemcpy(b->d_items, sorted.data(), sizeof(BatchItem) * sorted.size(), hipMemcpyHostToDevice));
  if (hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(ctx, QC_E_DEVICE, "stream"));
  for (int i = 0; i < N_BUCKET; ++i)
    if (hipStreamCreateWithFlags(&b->bs[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming) != hipSuccess)
      return bail(fail(ctx, QC_E_DEVICE, "stream"));
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess || hipEventCreate(&b->t0) != hipSuccess ||
      hipEventCreate(&b->t1) != hipSuccess)
    return bail(fail(ctx, QC_E_DEVICE, "event"));
  qc_status st = build_graph(b);
  if (st != QC_OK) return bail(st);
  *out = b;
  return QC_OK;
}

int32_t qc_batch_n_intervals(const qc_batch* b) { return b ? b->n_int : -1; }

qc_status qc_batch_ws_features(qc_batch* b, float* feat, int32_t feat_stride, double* chisq_unit, int32_t ref_ant,
                               void* stream) {
  if (!b) return QC_E_ARG;
  qc_ctx* ctx = b->ctx;
  if (!feat) return fail(ctx, QC_E_ARG, "feat is NULL");
  if (feat_stride < b->max_ant * 8)
    return fail(ctx, QC_E_ARG, "feat_stride %d is below 8 x the largest antenna count (%d)", feat_stride, b->max_ant);
  for (int i = 0; i < b->n_prob; ++i)
    if (ref_ant >= b->probs[i].vis.n_ant)
      return fail(ctx, QC_E_ARG, "ref_ant %d outside problem %d's %d antennas", ref_ant, i, b->probs[i].vis.n_ant);
  if (ws_features_lds(b->max_ant, 4) > 64 * 1024)
    return fail(ctx, QC_E_UNSUPPORTED, "features of %d antennas exceed the LDS budget", b->max_ant);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  HIP_TRY(ctx, launch_batch_features(b->d_probs, b->d_items, b->n_items, b->max_ant, b->vis_c128, feat, feat_stride,
                                     chisq_unit, ref_ant, s));
  return QC_OK;
}

qc_status qc_batch_ws_gains(qc_batch* b, const float* y, int32_t y_stride, void* stream) {
  if (!b) return QC_E_ARG;
  qc_ctx* ctx = b->ctx;
  if (!y) return fail(ctx, QC_E_ARG, "y is NULL");
  if (!b->all_diag) return fail(ctx, QC_E_UNSUPPORTED, "warm-start gains need DIAGONAL terms in every problem");
  if (y_stride < b->max_ant * 4)
    return fail(ctx, QC_E_ARG, "y_stride %d is below 4 x the largest antenna count (%d)", y_stride, b->max_ant);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  HIP_TRY(ctx, launch_batch_ws_gains(b->d_probs, b->d_items, b->n_items, b->max_ant, y, y_stride, s));
  return QC_OK;
}

qc_status qc_batch_run(qc_batch* b, void* stream) {
  if (!b) return QC_E_ARG;
  qc_ctx* ctx = b->ctx;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ctx->last_stream = s;
  // order the graph after earlier work on `stream` and later work after it
  HIP_TRY(ctx, hipEventRecord(b->t0, s));
  HIP_TRY(ctx, hipStreamWaitEvent(b->cs, b->t0, 0));
  HIP_TRY(ctx, hipGraphLaunch(b->exec, b->cs));
  HIP_TRY(ctx, hipEventRecord(b->t1, b->cs));
  HIP_TRY(ctx, hipStreamWaitEvent(s, b->t1, 0));
  ctx->timed = false;
  return QC_OK;
}

double qc_batch_last_ms(qc_batch* b) {
  if (!b) return -1.0;
  if (hipEventSynchronize(b->t1) != hipSuccess) return -1.0;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, b->t0, b->t1) != hipSuccess) return -1.0;
  return (double)ms;
}

qc_status qc_batch_tune(qc_batch* b, int32_t reps) {
  if (!b) return QC_E_ARG;
  qc_ctx* ctx = b->ctx;
  if (reps <= 0) reps = 1;
  // snapshot every problem's gains: each trial solves from the same start
  std::vector<size_t> gsz(b->n_prob);
  size_t total = 0;
  for (int i = 0; i < b->n_prob; ++i) {
    const qc_problem& P = b->problems[i];
    gsz[i] = (size_t)P.term.n_gt * P.term.n_gf * P.vis.n_ant * P.term.n_gdir * 4 * sizeof(double2);
    total += gsz[i];
  }
  unsigned char* snap = nullptr;
  HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&snap), std::max<size_t>(total, 1)));
  auto copy_all = [&](bool to_snap) -> hipError_t {
    size_t off = 0;
    for (int i = 0; i < b->n_prob; ++i) {
      void* g = b->problems[i].term.gains;
      hipError_t e = to_snap ? hipMemcpyAsync(snap + off, g, gsz[i], hipMemcpyDeviceToDevice, b->cs)
                             : hipMemcpyAsync(g, snap + off, gsz[i], hipMemcpyDeviceToDevice, b->cs);
      if (e != hipSuccess) return e;
      off += gsz[i];
    }
    return hipSuccess;
  };
  qc_status st = QC_OK;
  hipError_t e = copy_all(true);
  const int waves_c[] = {1, 2, 4, 8};
  const int rps_c[] = {1, 2, 4};
  for (int i = 0; i < N_BUCKET && e == hipSuccess && st == QC_OK; ++i) {
    Bucket& bk = b->bucket[i];
    if (bk.count == 0) continue;
    Bucket best = bk;
    best.ms = 1e30f;
    for (int w : waves_c) {
      for (int r : rps_c) {
        Bucket trial = bk;
        st = bucket_config(b, trial, w, r);
        if (st != QC_OK) break;
        const Bucket saved = bk;
        bk = trial;
        float best_rep = 1e30f;
        for (int k = 0; k < reps && e == hipSuccess; ++k) {
          e = copy_all(false);
          if (e == hipSuccess) e = launch_zero_ints(b->d_queue + i, 1, b->cs);
          if (e == hipSuccess) e = hipEventRecord(b->t0, b->cs);
          if (e == hipSuccess) {
            st = launch_bucket(b, i, b->cs);
            if (st != QC_OK) break;
          }
          if (e == hipSuccess) e = hipEventRecord(b->t1, b->cs);
          if (e == hipSuccess) e = hipEventSynchronize(b->t1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, b->t0, b->t1);
          best_rep = std::min(best_rep, ms);
        }
        bk = saved;
        if (st != QC_OK || e != hipSuccess) break;
        if (best_rep < best.ms) {
          best = trial;
          best.ms = best_rep;
        }
      }
      if (st != QC_OK || e != hipSuccess) break;
    }
    if (st == QC_OK && e == hipSuccess) bk = best;
  }
  if (e == hipSuccess) e = copy_all(false);
  if (e == hipSuccess) e = hipStreamSynchronize(b->cs);
  hipFree(snap);
  if (st != QC_OK) return st;
  if (e != hipSuccess) return fail(ctx, QC_E_DEVICE, "batch tune: %s", hipGetErrorString(e));
  return build_graph(b);
}

qc_status qc_batch_schedule(const qc_batch* b, int32_t* items, int32_t* waves, int32_t* rows_per_step,
                            float* tuned_ms, int32_t n) {
  if (!b || n < N_BUCKET) return QC_E_ARG;
  for (int i = 0; i < N_BUCKET; ++i) {
    if (items) items[i] = b->bucket[i].count;
    if (waves) waves[i] = b->bucket[i].waves;
    if (rows_per_step) rows_per_step[i] = b->bucket[i].rps;
    if (tuned_ms) tuned_ms[i] = b->bucket[i].ms;
  }
  return QC_OK;
}

qc_status qc_batch_destroy(qc_batch* b) {
  if (!b) return QC_E_ARG;
  hipSetDevice(b->ctx->device);
  if (b->cs) hipStreamSynchronize(b->cs);
  drop_graph(b);
  hipFree(b->d_probs);
  hipFree(b->d_items);
  hipFree(b->d_queue);
  for (int i = 0; i < N_BUCKET; ++i) {
    if (b->bs[i]) hipStreamDestroy(b->bs[i]);
    if (b->join[i]) hipEventDestroy(b->join[i]);
  }
  if (b->cs) hipStreamDestroy(b->cs);
  if (b->fork) hipEventDestroy(b->fork);
  if (b->t0) hipEventDestroy(b->t0);
  if (b->t1) hipEventDestroy(b->t1);
  delete b;
  return QC_OK;
}

qc_status qc_solve_batch(qc_ctx* ctx, const qc_problem* problems, int32_t n_problem, const qc_solve_opts* opts) {
  qc_batch* b = nullptr;
  qc_status st = qc_batch_create(ctx, problems, n_problem, opts, &b);
  if (st != QC_OK) return st;
  st = qc_batch_run(b, opts->stream);
  if (st == QC_OK) {
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(opts->stream));
    if (e != hipSuccess) st = fail(ctx, QC_E_DEVICE, "batch: %s", hipGetErrorString(e));
  }
  qc_batch_destroy(b);
  return st;
}

}  // extern "C"
