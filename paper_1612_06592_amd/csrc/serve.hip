// Serving loop: many observation streams, one device.
//
// One host thread owns all scheduling.  Each open stream has its carried
// state (overlap-save tail, synthesis history) and its chunk buffers
// resident in a caller-provided device arena and its own HIP stream.  A
// submitted block waits until a slot and arena space for its candidates
// and trigger workspace are free (admission), then runs as hop-aligned
// chunks of chunk_t samples; the loop always issues the next chunk of the
// admitted block with the earliest deadline, keeping at most two chunks of
// any stream queued on the device, so the work of different streams
// overlaps on the GPU and a block that arrives late but is due early is
// not stuck behind a long one.  The last chunk of a block also runs the
// trigger and copies the results to pinned host memory; the loop notices
// completion through an event and hands the result to lp_stream_poll.
//
// The simulated executor (lp_server_create_sim) replaces every device
// action by a completion time on one modelled in-order queue, so that the
// same loop can be exercised without a GPU.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>

#include "lp_internal.h"

namespace lp {

static int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

static size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Completion marker: a HIP event, or a modelled completion time.
struct Mark {
  hipEvent_t ev = nullptr;
  int64_t sim_done = 0;
};

struct Block {
  const void *x = nullptr;
  int64_t n_t = 0, frame0 = 0;
  uint64_t tag = 0;
  int32_t flags = 0;
  int64_t submit_ns = 0, deadline_ns = 0;
  size_t ws_off = 0, ws_bytes = 0;
  int next_chunk = 0, n_chunks = 0;
  bool final_issued = false;
  bool waited = false;       // counted once in admit_waits
  lp_status status = LP_OK;  // a launch failure of this block
  Mark done;
};

struct Stream {
  int id = 0;
  // Descriptor copies.
  std::vector<double> enu, tec;
  std::vector<float> gain;
  std::vector<int32_t> k;
  std::vector<lp_dir> beams;
  lp_array array{};
  lp_band band{};
  int n_beams = 0, n_tec = 0, dtype = 0, prec = 0, trig_cap = 0;
  float k_sigma = 6.0f;
  int64_t max_n_t = 0;
  double deadline_s = 0.0;
  // Plans (real executor).
  BfPlan *bf = nullptr;
  DdPlan *dd = nullptr;
  SynPlan *syn = nullptr;
  hipStream_t hs = nullptr;
  // Resident arena region: tail | hist | y chunk | d chunk.
  size_t res_off = 0, res_bytes = 0;
  size_t tail_off = 0, hist_off = 0, y_off = 0, d_off = 0;
  // Pinned host results of the block in flight.
  lp_trig *h_trig = nullptr;
  float *h_snr = nullptr;
  int32_t *h_best = nullptr;
  int32_t *h_n = nullptr;
  int64_t frame0 = 0;
  std::deque<Block> pending;
  bool active = false;
  Block cur;
  std::deque<Mark> chunk_marks;  // issued, not yet seen complete
  bool closing = false;
  int64_t station_beam_per_sample() const {
    return (int64_t)array.n_st * array.n_pol * band.n_sb * n_beams;
  }
};

struct ResultRec {
  lp_result r{};
  std::vector<lp_trig> trig;
  std::vector<float> snr;
  std::vector<int32_t> best;
};

}  // namespace lp

struct lp_server {
  lp_ctx *ctx = nullptr;
  bool sim = false;
  double sim_ns_per_sample = 0.0;
  int64_t sim_device_free = 0;
  char *arena_base = nullptr;
  lp::Arena arena;
  int max_slots = 16;
  int64_t chunk_t = 8192;
  int slots_used = 0;
  int next_id = 1;
  std::map<int, std::unique_ptr<lp::Stream>> streams;
  std::deque<lp::ResultRec> results;
  std::vector<lp::ResultRec> polled;  // storage behind the last poll
  std::mutex mu;
  std::condition_variable cv_work, cv_results;
  std::thread worker;
  bool stop = false;
  int64_t blocks_done = 0, chunks_issued = 0, admit_waits = 0;
  lp_status worker_error = LP_OK;
};

namespace lp {

static void sizes_of(const lp_stream_cfg *c, int64_t chunk_t, size_t *tail,
                     size_t *hist, size_t *y, size_t *d) {
  const int S = c->band.n_sb, B = c->n_beams, J = c->n_tec;
  *tail = align256((size_t)B * S * kHist * 8);
  *hist = align256((size_t)B * J * S * kSynHist * 8);
  *y = align256((size_t)B * S * chunk_t * 8);
  *d = align256((size_t)B * J * S * chunk_t * 8);
}

struct BlockLayout {
  size_t cand, work, trig, n, snr, best, total;
};

static BlockLayout block_layout(const lp_stream_cfg *c, int64_t n_t,
                                int trig_cap) {
  const int B = c->n_beams, J = c->n_tec;
  BlockLayout L;
  size_t o = 0;
  L.cand = o;
  o += align256(lp_cand_bytes(B * J, n_t));
  L.work = o;
  o += align256(lp_trigger_work_bytes(B, J, n_t));
  L.trig = o;
  o += align256((size_t)trig_cap * sizeof(lp_trig));
  L.n = o;
  o += 256;
  L.snr = o;
  o += align256((size_t)B * J * 4);
  L.best = o;
  o += align256((size_t)B * 4);
  L.total = o;
  return L;
}

static int trig_cap_of(const lp_stream_cfg *c) {
  return c->trig_cap > 0 ? c->trig_cap : 1024;
}

static bool mark_done(lp_server *s, const Mark &m, lp_status *err) {
  if (s->sim) return now_ns() >= m.sim_done;
  hipError_t e = hipEventQuery(m.ev);
  if (e == hipSuccess) return true;
  if (e == hipErrorNotReady) return false;
  *err = hip_fail(e, "hipEventQuery");
  return true;
}

static lp_status new_mark(lp_server *s, Stream *st, int64_t cost_ns, Mark *m) {
  if (s->sim) {
    int64_t t = std::max(now_ns(), s->sim_device_free) + cost_ns;
    s->sim_device_free = t;
    m->sim_done = t;
    return LP_OK;
  }
  LP_HIP(hipEventCreateWithFlags(&m->ev, hipEventDisableTiming));
  LP_HIP(hipEventRecord(m->ev, st->hs));
  return LP_OK;
}

static void free_mark(lp_server *s, Mark &m) {
  if (!s->sim && m.ev) (void)hipEventDestroy(m.ev);
  m.ev = nullptr;
}

// Issue the next chunk of st->cur (lock held).
static lp_status issue_chunk(lp_server *s, Stream *st) {
  Block &b = st->cur;
  const int64_t t0 = (int64_t)b.next_chunk * s->chunk_t;
  const int64_t c = std::min<int64_t>(s->chunk_t, b.n_t - t0);
  const bool last = (b.next_chunk + 1 == b.n_chunks);
  const int B = st->n_beams, J = st->n_tec, S = st->band.n_sb;
  int64_t cost = (int64_t)(s->sim_ns_per_sample *
                           (double)st->station_beam_per_sample() * (double)c *
                           std::max(1, J));
  if (!s->sim) {
    char *A = s->arena_base;
    char *ws = A + b.ws_off;
    BlockLayout L;
    {
      lp_stream_cfg cfg{};
      cfg.n_beams = B;
      cfg.n_tec = J;
      cfg.band = st->band;
      L = block_layout(&cfg, b.n_t, st->trig_cap);
    }
    if (b.next_chunk == 0 && (b.flags & LP_SUBMIT_RESET)) {
      LP_HIP(hipMemsetAsync(A + st->tail_off, 0, (size_t)B * S * kHist * 8,
                            st->hs));
      LP_HIP(hipMemsetAsync(A + st->hist_off, 0,
                            (size_t)B * J * S * kSynHist * 8, st->hs));
    }
    lp_status rc;
    if ((rc = bf_launch(st->bf, b.x, st->dtype, b.n_t, t0, c, S,
                        A + st->y_off, st->hs)))
      return rc;
    if ((rc = dd_launch(s->ctx, st->dd, S, A + st->y_off, B, c,
                        A + st->tail_off, true, A + st->d_off, 0, J, st->hs)))
      return rc;
    if ((rc = syn_launch(s->ctx, st->syn, S, A + st->d_off, B * J, c,
                         b.frame0 + t0, A + st->hist_off, nullptr,
                         ws + L.cand, b.n_t, t0, 0, B * J, st->hs)))
      return rc;
    if (last) {
      if ((rc = trig_launch(ws + L.cand, B, J, b.n_t, b.frame0, st->k_sigma,
                            reinterpret_cast<lp_trig *>(ws + L.trig),
                            st->trig_cap, reinterpret_cast<int *>(ws + L.n),
                            reinterpret_cast<float *>(ws + L.snr),
                            reinterpret_cast<int *>(ws + L.best), nullptr,
                            ws + L.work, st->hs)))
        return rc;
      LP_HIP(hipMemcpyAsync(st->h_n, ws + L.n, 4, hipMemcpyDeviceToHost,
                            st->hs));
      LP_HIP(hipMemcpyAsync(st->h_trig, ws + L.trig,
                            (size_t)st->trig_cap * sizeof(lp_trig),
                            hipMemcpyDeviceToHost, st->hs));
      LP_HIP(hipMemcpyAsync(st->h_snr, ws + L.snr, (size_t)B * J * 4,
                            hipMemcpyDeviceToHost, st->hs));
      LP_HIP(hipMemcpyAsync(st->h_best, ws + L.best, (size_t)B * 4,
                            hipMemcpyDeviceToHost, st->hs));
    }
  }
  Mark m;
  lp_status rc = new_mark(s, st, cost, &m);
  if (rc) return rc;
  b.next_chunk++;
  s->chunks_issued++;
  if (last) {
    b.done = m;
    if (!s->sim) {
      // The chunk list keeps its own event for the queue-depth count.
      Mark m2;
      if ((rc = new_mark(s, st, 0, &m2))) return rc;
      st->chunk_marks.push_back(m2);
    } else {
      st->chunk_marks.push_back(m);
    }
    b.final_issued = true;
  } else {
    st->chunk_marks.push_back(m);
  }
  return LP_OK;
}

static void push_result(lp_server *s, Stream *st, const Block &b,
                        lp_status status) {
  ResultRec rec;
  lp_result &r = rec.r;
  r.stream = st->id;
  r.status = status;
  r.tag = b.tag;
  r.n_t = b.n_t;
  r.frame0 = b.frame0;
  r.n_beams = st->n_beams;
  r.n_tec = st->n_tec;
  r.submit_ns = b.submit_ns;
  r.done_ns = now_ns();
  r.latency_ns = r.done_ns - b.submit_ns;
  r.deadline_ns = b.deadline_ns - b.submit_ns;
  if (status == LP_OK && !s->sim) {
    int n = *st->h_n;
    r.n_trig = n;
    rec.trig.assign(st->h_trig, st->h_trig + std::min(n, st->trig_cap));
    rec.snr.assign(st->h_snr, st->h_snr + st->n_beams * st->n_tec);
    rec.best.assign(st->h_best, st->h_best + st->n_beams);
  } else {
    rec.snr.assign((size_t)st->n_beams * st->n_tec, 0.0f);
    rec.best.assign(st->n_beams, 0);
  }
  s->results.push_back(std::move(rec));
  s->cv_results.notify_all();
}

// Device-side resources of a stream other than its arena space: its HIP
// stream, pinned result buffers and its holds on the plans.
static void drop_device_side(lp_server *s, Stream *st) {
  if (s->sim) return;
  if (st->hs) (void)hipStreamSynchronize(st->hs);
  for (auto &m : st->chunk_marks) free_mark(s, m);
  if (st->hs) (void)hipStreamDestroy(st->hs);
  st->hs = nullptr;
  if (st->h_trig) (void)hipHostFree(st->h_trig);
  if (st->h_snr) (void)hipHostFree(st->h_snr);
  if (st->h_best) (void)hipHostFree(st->h_best);
  if (st->h_n) (void)hipHostFree(st->h_n);
  st->h_trig = nullptr;
  st->h_snr = nullptr;
  st->h_best = nullptr;
  st->h_n = nullptr;
  if (st->bf) plan_release(s->ctx, st->bf);
  if (st->dd) plan_release(s->ctx, st->dd);
  if (st->syn) plan_release(s->ctx, st->syn);
  st->bf = nullptr;
  st->dd = nullptr;
  st->syn = nullptr;
}

static void release_stream(lp_server *s, Stream *st) {
  drop_device_side(s, st);
  st->chunk_marks.clear();
  s->arena.release(st->res_off, st->res_bytes);
}

// One pass of the loop (lock held).  Returns true if it changed anything.
static bool step(lp_server *s) {
  bool progress = false;
  lp_status err = LP_OK;
  // 1. Retire finished chunks and blocks.
  for (auto &kv : s->streams) {
    Stream *st = kv.second.get();
    while (!st->chunk_marks.empty() &&
           mark_done(s, st->chunk_marks.front(), &err)) {
      if (!s->sim && st->chunk_marks.front().ev != st->cur.done.ev)
        free_mark(s, st->chunk_marks.front());
      st->chunk_marks.pop_front();
      progress = true;
    }
    if (st->active && st->cur.final_issued && mark_done(s, st->cur.done, &err)) {
      push_result(s, st, st->cur, st->cur.status ? st->cur.status : err);
      free_mark(s, st->cur.done);
      s->arena.release(st->cur.ws_off, st->cur.ws_bytes);
      st->active = false;
      s->slots_used--;
      s->blocks_done++;
      progress = true;
    }
  }
  // 2. Closing streams: drop queued blocks, release once idle.
  for (auto it = s->streams.begin(); it != s->streams.end();) {
    Stream *st = it->second.get();
    if (st->closing) {
      while (!st->pending.empty()) {
        push_result(s, st, st->pending.front(), LP_ECLOSED);
        st->pending.pop_front();
        progress = true;
      }
      if (!st->active && st->chunk_marks.empty()) {
        release_stream(s, st);
        it = s->streams.erase(it);
        progress = true;
        continue;
      }
    }
    ++it;
  }
  // 3. Admission: earliest-deadline queued block first.
  for (;;) {
    Stream *pick = nullptr;
    for (auto &kv : s->streams) {
      Stream *st = kv.second.get();
      if (st->active || st->closing || st->pending.empty()) continue;
      if (!pick || st->pending.front().deadline_ns <
                       pick->pending.front().deadline_ns)
        pick = st;
    }
    if (!pick || s->slots_used >= s->max_slots) break;
    Block &front = pick->pending.front();
    lp_stream_cfg cfg{};
    cfg.n_beams = pick->n_beams;
    cfg.n_tec = pick->n_tec;
    cfg.band = pick->band;
    front.ws_bytes = block_layout(&cfg, front.n_t, pick->trig_cap).total;
    if (!s->arena.alloc(front.ws_bytes, &front.ws_off)) {
      if (!front.waited) s->admit_waits++;
      front.waited = true;
      break;
    }
    Block b = front;
    pick->pending.pop_front();
    if (b.flags & LP_SUBMIT_RESET) pick->frame0 = 0;
    b.frame0 = pick->frame0;
    pick->frame0 += b.n_t;
    b.n_chunks = (int)((b.n_t + s->chunk_t - 1) / s->chunk_t);
    pick->cur = b;
    pick->active = true;
    s->slots_used++;
    progress = true;
  }
  // 4. Issue chunks, earliest deadline first, at most two queued per stream.
  for (;;) {
    Stream *pick = nullptr;
    for (auto &kv : s->streams) {
      Stream *st = kv.second.get();
      if (!st->active || st->cur.next_chunk >= st->cur.n_chunks) continue;
      if (st->chunk_marks.size() >= 2) continue;
      if (!pick || st->cur.deadline_ns < pick->cur.deadline_ns) pick = st;
    }
    if (!pick) break;
    lp_status rc = issue_chunk(s, pick);
    if (rc) {
      // A failed launch finishes the block with that status.
      s->worker_error = rc;
      pick->cur.status = rc;
      pick->cur.next_chunk = pick->cur.n_chunks;
      pick->cur.final_issued = true;
      if (new_mark(s, pick, 0, &pick->cur.done) != LP_OK)
        pick->cur.done.sim_done = 0, pick->cur.done.ev = nullptr;
    }
    progress = true;
  }
  return progress;
}

static void loop(lp_server *s) {
  if (!s->sim) (void)hipSetDevice(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progress = step(s);
    bool busy = false;
    for (auto &kv : s->streams)
      if (kv.second->active || !kv.second->chunk_marks.empty()) busy = true;
    if (s->stop && !busy) {
      bool queued = false;
      for (auto &kv : s->streams) queued |= !kv.second->pending.empty();
      if (!queued) break;
    }
    if (progress) continue;
    if (busy)
      s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    else
      s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
  }
}

static lp_status check_cfg(const lp_stream_cfg *c) {
  if (!c) return set_error(LP_EINVAL, "stream cfg is NULL");
  lp_status rc = check_band(&c->band);
  if (rc) return rc;
  if (c->array.n_st <= 0 || c->array.n_pol <= 0 || !c->array.enu_m)
    return set_error(LP_EINVAL, "stream cfg: bad array");
  if (c->array.n_st * c->array.n_pol > 128)
    return set_error(LP_EINVAL, "stream cfg: more than 128 inputs");
  if (c->n_beams <= 0 || c->n_beams > 64 || !c->beams)
    return set_error(LP_EINVAL, "stream cfg: n_beams must be 1..64");
  if (c->n_tec <= 0 || c->n_tec > 4096 || !c->tec_tecu)
    return set_error(LP_EINVAL, "stream cfg: bad TEC list");
  for (int j = 0; j < c->n_tec; ++j)
    if (!(c->tec_tecu[j] >= 0.0 && c->tec_tecu[j] <= 1000.0))
      return set_error(LP_EINVAL, "stream cfg: TEC outside [0, 1000]");
  if (c->dtype != LP_CI8 && c->dtype != LP_CI16)
    return set_error(LP_EINVAL, "stream cfg: dtype");
  if (c->prec != LP_FP32 && c->prec != LP_FP16_MFMA)
    return set_error(LP_EINVAL, "stream cfg: precision");
  if (const char *why = bf_shape_error(c->array.n_st * c->array.n_pol,
                                       c->dtype, c->prec))
    return set_error(LP_EINVAL, "stream cfg: %s", why);
  if (c->max_n_t <= 0 || c->max_n_t % kHop)
    return set_error(LP_EINVAL, "stream cfg: max_n_t must be a multiple of %d",
                     kHop);
  if (!(c->k_sigma > 0.0f))
    return set_error(LP_EINVAL, "stream cfg: k_sigma must be positive");
  if (check_trigger_args(c->n_beams, c->n_tec, c->max_n_t, 0, c->k_sigma, 0))
    return set_error(LP_EINVAL, "stream cfg: trigger limits (%s)",
                     lp_last_error());
  if (c->trig_cap < 0) return set_error(LP_EINVAL, "stream cfg: trig_cap");
  return LP_OK;
}

static lp_status create(lp_ctx *ctx, bool sim, double ns_per_sample,
                        void *arena, size_t arena_bytes, int32_t max_slots,
                        int64_t chunk_t, lp_server **out) {
  if (!out) return set_error(LP_EINVAL, "out is NULL");
  *out = nullptr;
  if (chunk_t == 0) chunk_t = 8192;
  if (chunk_t < 0 || chunk_t % kHop)
    return set_error(LP_EINVAL, "chunk_t must be a multiple of %d", kHop);
  if (max_slots < 0 || max_slots > 4096)
    return set_error(LP_EINVAL, "max_slots %d", max_slots);
  auto s = std::make_unique<lp_server>();
  s->ctx = ctx;
  s->sim = sim;
  s->sim_ns_per_sample = ns_per_sample;
  s->arena_base = static_cast<char *>(arena);
  s->arena.init(arena_bytes);
  s->max_slots = max_slots ? max_slots : 16;
  s->chunk_t = chunk_t;
  lp_server *raw = s.release();
  raw->worker = std::thread(loop, raw);
  *out = raw;
  return LP_OK;
}

}  // namespace lp

using namespace lp;

extern "C" {

size_t lp_stream_resident_bytes(const lp_stream_cfg *cfg, int64_t chunk_t) {
  if (!cfg) return 0;
  size_t a, b, c, d;
  sizes_of(cfg, chunk_t ? chunk_t : 8192, &a, &b, &c, &d);
  return a + b + c + d;
}

size_t lp_block_bytes(const lp_stream_cfg *cfg, int64_t n_t) {
  if (!cfg) return 0;
  return block_layout(cfg, n_t, trig_cap_of(cfg)).total;
}

lp_status lp_server_create(lp_ctx *ctx, void *arena_dev, size_t arena_bytes,
                           int32_t max_slots, int64_t chunk_t,
                           lp_server **out) {
  if (!ctx || !arena_dev || !arena_bytes)
    return set_error(LP_EINVAL, "lp_server_create: NULL ctx or arena");
  if (reinterpret_cast<uintptr_t>(arena_dev) % 256)
    return set_error(LP_EINVAL, "lp_server_create: arena must be 256-byte "
                                "aligned");
  return create(ctx, false, 0.0, arena_dev, arena_bytes, max_slots, chunk_t,
                out);
}

lp_status lp_server_create_sim(double ns_per_sample, size_t arena_bytes,
                               int32_t max_slots, int64_t chunk_t,
                               lp_server **out) {
  if (!(ns_per_sample >= 0.0) || !arena_bytes)
    return set_error(LP_EINVAL, "lp_server_create_sim: bad model or arena");
  return create(nullptr, true, ns_per_sample, nullptr, arena_bytes, max_slots,
                chunk_t, out);
}

lp_status lp_stream_open(lp_server *srv, const lp_stream_cfg *cfg,
                         int32_t *id) {
  if (!srv || !id) return set_error(LP_EINVAL, "lp_stream_open: NULL");
  lp_status rc = check_cfg(cfg);
  if (rc) return rc;
  auto st = std::make_unique<Stream>();
  st->enu.assign(cfg->array.enu_m, cfg->array.enu_m + 3 * cfg->array.n_st);
  const int n_in = cfg->array.n_st * cfg->array.n_pol;
  if (cfg->array.gain) st->gain.assign(cfg->array.gain, cfg->array.gain + n_in);
  st->k.assign(cfg->band.k, cfg->band.k + cfg->band.n_sb);
  st->beams.assign(cfg->beams, cfg->beams + cfg->n_beams);
  st->tec.assign(cfg->tec_tecu, cfg->tec_tecu + cfg->n_tec);
  st->array = cfg->array;
  st->array.enu_m = st->enu.data();
  st->array.gain = st->gain.empty() ? nullptr : st->gain.data();
  st->band = cfg->band;
  st->band.k = st->k.data();
  st->n_beams = cfg->n_beams;
  st->n_tec = cfg->n_tec;
  st->dtype = cfg->dtype;
  st->prec = cfg->prec;
  st->k_sigma = cfg->k_sigma;
  st->max_n_t = cfg->max_n_t;
  st->trig_cap = trig_cap_of(cfg);
  st->deadline_s = cfg->deadline_s;
  size_t tail, hist, y, d;
  sizes_of(cfg, srv->chunk_t, &tail, &hist, &y, &d);
  st->res_bytes = tail + hist + y + d;
  if (!srv->sim) {
    // The stream's HIP stream first: its plans' tables are written there,
    // outside the server lock; the stream holds the plans until it closes.
    if ((rc = set_device(srv->ctx))) return rc;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&st->hs, hipStreamNonBlocking)))
      return hip_fail(e, "hipStreamCreate");
    auto undo = [&](lp_status r) {
      drop_device_side(srv, st.get());
      return r;
    };
    {
      PlanRef<BfPlan> bf;
      PlanRef<DdPlan> dd;
      PlanRef<SynPlan> syn;
      if ((rc = get_bf_plan(srv->ctx, &st->array, &st->band, st->beams.data(),
                            st->n_beams, st->prec, st->dtype, st->hs, bf)) ||
          (rc = get_dd_plan(srv->ctx, &st->band, st->tec.data(), st->n_tec,
                            st->hs, dd)) ||
          (rc = get_syn_plan(srv->ctx, &st->band, st->hs, syn)))
        return undo(rc);
      st->bf = bf.keep();
      st->dd = dd.keep();
      st->syn = syn.keep();
    }
    if ((e = hipHostMalloc((void **)&st->h_trig,
                           (size_t)st->trig_cap * sizeof(lp_trig))) ||
        (e = hipHostMalloc((void **)&st->h_snr,
                           (size_t)st->n_beams * st->n_tec * 4)) ||
        (e = hipHostMalloc((void **)&st->h_best, (size_t)st->n_beams * 4)) ||
        (e = hipHostMalloc((void **)&st->h_n, 16)))
      return undo(hip_fail(e, "hipHostMalloc"));
  }
  std::unique_lock<std::mutex> lk(srv->mu);
  if (srv->stop) {
    drop_device_side(srv, st.get());
    return set_error(LP_ECLOSED, "server is shutting down");
  }
  if (!srv->arena.alloc(st->res_bytes, &st->res_off)) {
    drop_device_side(srv, st.get());
    return set_error(LP_EAGAIN,
                     "lp_stream_open: %zu resident bytes do not fit the "
                     "arena now", st->res_bytes);
  }
  st->tail_off = st->res_off;
  st->hist_off = st->tail_off + tail;
  st->y_off = st->hist_off + hist;
  st->d_off = st->y_off + y;
  if (!srv->sim) {
    hipError_t e;
    char *A = srv->arena_base;
    if ((e = hipMemsetAsync(A + st->tail_off, 0, tail + hist, st->hs)) ||
        (e = hipStreamSynchronize(st->hs))) {
      srv->arena.release(st->res_off, st->res_bytes);
      drop_device_side(srv, st.get());
      return hip_fail(e, "hipMemset(state)");
    }
  }
  st->id = srv->next_id++;
  *id = st->id;
  srv->streams[st->id] = std::move(st);
  return LP_OK;
}

lp_status lp_stream_submit(lp_server *srv, int32_t id, const void *block,
                           int64_t n_t, uint64_t tag, int32_t flags) {
  if (!srv) return set_error(LP_EINVAL, "lp_stream_submit: NULL server");
  if (flags & ~LP_SUBMIT_RESET)
    return set_error(LP_EINVAL, "lp_stream_submit: unknown flags");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->streams.find(id);
  if (it == srv->streams.end())
    return set_error(LP_EINVAL, "lp_stream_submit: no stream %d", id);
  Stream *st = it->second.get();
  if (st->closing || srv->stop)
    return set_error(LP_ECLOSED, "lp_stream_submit: stream %d is closing", id);
  if (n_t <= 0 || n_t % kHop || n_t > st->max_n_t)
    return set_error(LP_EINVAL,
                     "lp_stream_submit: n_t %lld not a positive multiple of "
                     "%d up to %lld", (long long)n_t, kHop,
                     (long long)st->max_n_t);
  if (!srv->sim && (!block || reinterpret_cast<uintptr_t>(block) % 16))
    return set_error(LP_EINVAL, "lp_stream_submit: block must be 16-byte "
                                "aligned device memory");
  Block b;
  b.x = block;
  b.n_t = n_t;
  b.tag = tag;
  b.flags = flags;
  b.submit_ns = now_ns();
  const double dur = (double)n_t * kM / st->band.fs_hz;
  const double budget = st->deadline_s > 0 ? st->deadline_s : 5.0 - dur;
  b.deadline_ns = b.submit_ns + (int64_t)(budget * 1e9);
  st->pending.push_back(b);
  srv->cv_work.notify_all();
  return LP_OK;
}

lp_status lp_stream_poll(lp_server *srv, lp_result *out, int32_t cap,
                         int32_t *n, int32_t timeout_us) {
  if (!srv || !n || (cap > 0 && !out))
    return set_error(LP_EINVAL, "lp_stream_poll: NULL argument");
  *n = 0;
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->polled.clear();
  if (srv->results.empty() && timeout_us > 0)
    srv->cv_results.wait_for(lk, std::chrono::microseconds(timeout_us),
                             [&] { return !srv->results.empty(); });
  while (*n < cap && !srv->results.empty()) {
    srv->polled.push_back(std::move(srv->results.front()));
    srv->results.pop_front();
    ++*n;
  }
  for (int i = 0; i < *n; ++i) {
    ResultRec &r = srv->polled[i];
    r.r.trig = r.trig.data();
    r.r.snr = r.snr.data();
    r.r.best_tec = r.best.data();
    out[i] = r.r;
  }
  if (*n == 0) return set_error(LP_ETIMEOUT, "lp_stream_poll: no results");
  return LP_OK;
}

lp_status lp_stream_close(lp_server *srv, int32_t id) {
  if (!srv) return set_error(LP_EINVAL, "lp_stream_close: NULL server");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->streams.find(id);
  if (it == srv->streams.end() || it->second->closing)
    return set_error(LP_EINVAL, "lp_stream_close: no open stream %d", id);
  it->second->closing = true;
  srv->cv_work.notify_all();
  return LP_OK;
}

void lp_server_destroy(lp_server *srv) {
  if (!srv) return;
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->stop = true;
    for (auto &kv : srv->streams) kv.second->closing = true;
    srv->cv_work.notify_all();
  }
  if (srv->worker.joinable()) srv->worker.join();
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    for (auto &kv : srv->streams) release_stream(srv, kv.second.get());
    srv->streams.clear();
  }
  delete srv;
}

lp_status lp_server_stats(lp_server *srv, int64_t *blocks_done,
                          int64_t *chunks_issued, int64_t *admit_waits) {
  if (!srv) return set_error(LP_EINVAL, "lp_server_stats: NULL server");
  std::unique_lock<std::mutex> lk(srv->mu);
  if (blocks_done) *blocks_done = srv->blocks_done;
  if (chunks_issued) *chunks_issued = srv->chunks_issued;
  if (admit_waits) *admit_waits = srv->admit_waits;
  return srv->worker_error;
}

}  // extern "C"
