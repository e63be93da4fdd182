// Host-side stress of the serving loop on the simulated executor: several
// submitter threads, one poller, streams opened and closed while blocks are
// in flight.  Built with AddressSanitizer/UBSan or ThreadSanitizer (host
// code only) by tests/test_serve_sanitizers.py; exits non-zero on any
// lost, duplicated or misordered result.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/lp.h"

static void fail(const char *what) {
  std::fprintf(stderr, "serve_stress: %s (%s)\n", what, lp_last_error());
  std::exit(1);
}

int main() {
  lp_server *srv = nullptr;
  if (lp_server_create_sim(0.05, (size_t)1 << 34, 8, 4096, &srv)) fail("create");
  double enu[4 * 3] = {0};
  int32_t k[16];
  for (int i = 0; i < 16; ++i) k[i] = 60 + i;
  lp_dir beams[2] = {{0.1, 0.6}, {0.11, 0.6}};
  double tec[2] = {1.0, 2.0};
  lp_stream_cfg cfg{};
  cfg.array = {4, 2, enu, nullptr};
  cfg.band = {16, k, 100e6, 200e6, LP_M, LP_TAPS, 9.0};
  cfg.beams = beams;
  cfg.n_beams = 2;
  cfg.tec_tecu = tec;
  cfg.n_tec = 2;
  cfg.dtype = LP_CI8;
  cfg.prec = LP_FP16_MFMA;
  cfg.k_sigma = 6.0f;
  cfg.max_n_t = 16384;
  const int n_streams = 6, per_stream = 40;
  std::vector<int32_t> ids(n_streams);
  for (int i = 0; i < n_streams; ++i)
    if (lp_stream_open(srv, &cfg, &ids[i])) fail("open");
  std::atomic<int> submitted{0};
  std::vector<std::thread> th;
  for (int i = 0; i < n_streams; ++i)
    th.emplace_back([&, i] {
      for (int b = 0; b < per_stream; ++b) {
        int64_t n_t = 2048 * (1 + (b * 7 + i) % 8);
        if (lp_stream_submit(srv, ids[i], nullptr, n_t, (uint64_t)b, 0))
          fail("submit");
        submitted++;
      }
    });
  std::map<int, std::vector<uint64_t>> got;
  int n_results = 0;
  lp_result res[32];
  while (n_results < n_streams * per_stream) {
    int32_t n = 0;
    lp_status rc = lp_stream_poll(srv, res, 32, &n, 200000);
    if (rc == LP_ETIMEOUT) continue;
    if (rc) fail("poll");
    for (int j = 0; j < n; ++j) {
      if (res[j].status != LP_OK) fail("status");
      if (res[j].n_beams != 2 || res[j].n_tec != 2 || !res[j].snr) fail("shape");
      got[res[j].stream].push_back(res[j].tag);
    }
    n_results += n;
  }
  for (auto &t : th) t.join();
  for (auto &kv : got) {
    if ((int)kv.second.size() != per_stream) fail("count");
    for (int b = 0; b < per_stream; ++b)
      if (kv.second[b] != (uint64_t)b) fail("order");
  }
  // Close some streams with work queued, reopen, and tear down with work
  // in flight.
  for (int i = 0; i < n_streams; ++i)
    for (int b = 0; b < 4; ++b) lp_stream_submit(srv, ids[i], nullptr, 16384, 99, 0);
  for (int i = 0; i < n_streams; i += 2)
    if (lp_stream_close(srv, ids[i])) fail("close");
  int32_t again = 0;
  for (int tries = 0; tries < 1000 && lp_stream_open(srv, &cfg, &again); ++tries)
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  lp_server_destroy(srv);
  std::printf("serve_stress: ok (%d results)\n", n_results);
  return 0;
}
