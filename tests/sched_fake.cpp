// CPU tests of the serving scheduler (paper_2010_08735_amd/csrc/bh_sched.h) with a fake
// backend: launches "run" on a virtual clock, one after another like a stream, taking
// per_launch + per_tile * tiles seconds, and may be scripted to fail; images are fake
// addresses inside a byte budget.  Every scenario checks its own outcome and prints one
// line; the process exits non-zero on the first failed check.  Built with g++ by
// tests/test_sched_fake.py, plain and under ASan + UBSan and TSan.
//
//   sched_fake <scenario>      (scenario "all" runs every one)
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "bh_sched.h"

using namespace bh::sched;

#define CHECK(cond)                                                                    \
  do {                                                                                 \
    if (!(cond)) {                                                                     \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond);    \
      std::exit(1);                                                                    \
    }                                                                                  \
  } while (0)

struct Frame {
  int64_t tiles = 1;
  int id = 0;
};

struct PieceRec {
  uint64_t ticket;
  int64_t first, count;
};

struct LaunchRec {
  int64_t id;
  double start, end;
  int status;
  const void* group;
  std::vector<PieceRec> pieces;
};

// ---- virtual-clock backend ---------------------------------------------------------------
struct FakeBackend {
  using Payload = Frame;
  struct Handle {
    int64_t id = -1;
  };
  double t = 0;                  // virtual time (s)
  double per_launch = 10e-6, per_tile = 1e-6;
  double stream_free = 0;        // the device runs launches one after another
  std::map<int64_t, double> end; // launch id -> completion time
  int64_t next_id = 0;
  std::set<int64_t> fail;        // launch ids scripted to fail
  size_t budget = SIZE_MAX, used = 0, peak_used = 0;
  std::map<uintptr_t, size_t> live;
  uintptr_t next_addr = 0x10000;
  std::vector<LaunchRec> log;
  int in_flight = 0, peak_in_flight = 0;

  double now() { return t; }
  int64_t tiles(const Frame& f) { return f.tiles; }
  void* try_alloc(size_t bytes) {
    if (used + bytes > budget) return nullptr;
    used += bytes;
    peak_used = std::max(peak_used, used);
    uintptr_t a = next_addr;
    next_addr += 0x1000;
    live[a] = bytes;
    return (void*)a;
  }
  void dealloc(void* p, size_t bytes) {
    auto it = live.find((uintptr_t)p);
    CHECK(it != live.end() && it->second == bytes);
    live.erase(it);
    used -= bytes;
  }
  int launch(const std::vector<Piece<Frame>>& pieces, int64_t ntiles, Handle* h) {
    h->id = next_id++;
    const bool bad = fail.count(h->id) != 0;
    const double start = std::max(t, stream_free);
    const double e = start + (bad ? 0.0 : per_launch + per_tile * (double)ntiles);
    end[h->id] = e;
    stream_free = e;
    LaunchRec rec{h->id, start, e, bad ? kEDEVICE : kOK, pieces.empty() ? nullptr : pieces[0].r->group, {}};
    for (const auto& pc : pieces) {
      CHECK(pc.r->group == rec.group);
      CHECK(pc.count > 0);
      rec.pieces.push_back(PieceRec{pc.r->ticket, pc.first, pc.count});
    }
    log.push_back(rec);
    in_flight++;
    peak_in_flight = std::max(peak_in_flight, in_flight);
    return bad ? kEDEVICE : kOK;
  }
  bool done(Handle& h) { return t >= end.at(h.id); }
  void wait(Handle& h) { t = std::max(t, end.at(h.id)); }
  void release(Handle& h) {
    CHECK(t >= end.at(h.id));
    in_flight--;
  }
  // the next completion after t (or infinity)
  double next_end() const {
    double best = 1e300;
    for (auto& kv : end)
      if (kv.second > t) best = std::min(best, kv.second);
    return best;
  }
};

using Sched = Scheduler<FakeBackend>;

struct Arrival {
  double t;
  Frame f;
  const void* group;
  bool library_image;
  size_t bytes;
};

static int g_group_a, g_group_b;  // two table sets

// Drive the scheduler on the virtual clock: submit arrivals on time, step, and advance the
// clock to the next event when it asks to wait.  on_tick(t) may act as a client (poll,
// release) after every step.  Returns the tickets in arrival order.
static std::vector<uint64_t> drive(Sched& s, FakeBackend& b, const std::vector<Arrival>& arr,
                                   const std::function<void()>& on_tick = nullptr,
                                   double t_stop = 1e300, std::vector<int>* submit_rc = nullptr) {
  std::vector<uint64_t> tickets;
  size_t next = 0;
  bool stopped = false;
  for (int guard = 0; guard < 10000000; ++guard) {
    while (next < arr.size() && arr[next].t <= b.t) {
      uint64_t tk = 0;
      const Arrival& a = arr[next];
      int rc = s.submit(a.f, a.group, a.library_image ? nullptr : (float*)(uintptr_t)(0x7000000 + 64 * next),
                        a.bytes, &tk);
      if (submit_rc) submit_rc->push_back(rc);
      tickets.push_back(rc == kOK ? tk : 0);
      ++next;
    }
    if (!stopped && b.t >= t_stop) {
      s.stop();
      stopped = true;
    }
    Next n = s.step();
    if (on_tick) on_tick();
    if (n == Next::kStop) return tickets;
    if (n == Next::kAgain) continue;
    if (n == Next::kWaitOldest) {
      // clients keep submitting while the scheduler thread waits
      if (next < arr.size() && arr[next].t < b.next_end()) {
        b.t = std::max(b.t, arr[next].t);
        continue;
      }
      s.wait_oldest();
      continue;
    }
    // idle or polling: jump to the next arrival, completion or stop time
    double tn = std::min(b.next_end(), next < arr.size() ? arr[next].t : 1e300);
    if (!stopped) tn = std::min(tn, t_stop);
    if (tn >= 1e299) {
      if (next >= arr.size() && s.pending() == 0 && !stopped) {
        s.stop();
        stopped = true;
        continue;
      }
      if (on_tick) {  // a client may still free images
        b.t += 1e-3;
        continue;
      }
      CHECK(!"scheduler waits for nothing");
    }
    b.t = std::max(b.t, tn);
  }
  CHECK(!"scenario did not end");
  return tickets;
}

static Arrival arrival(double t, int64_t tiles, int id, const void* g = &g_group_a,
                       bool lib = false, size_t bytes = 1000) {
  return Arrival{t, Frame{tiles, id}, g, lib, bytes};
}

// ---- scenarios ---------------------------------------------------------------------------

// Equal frames submitted together complete in submission order, each with the launch that
// holds its last tile, and every tile is rendered exactly once.
static void fifo_order() {
  FakeBackend b;
  Params p;
  p.max_tiles = 8;
  Sched s(b, p);
  std::vector<Arrival> arr;
  for (int i = 0; i < 10; ++i) arr.push_back(arrival(0.0, 5, i));
  auto tk = drive(s, b, arr);
  std::map<uint64_t, int64_t> covered;
  for (auto& L : b.log)
    for (auto& pc : L.pieces) {
      CHECK(pc.first == covered[pc.ticket]);  // tiles in order, no gap, no overlap
      covered[pc.ticket] += pc.count;
    }
  double prev = -1;
  for (uint64_t t : tk) {
    int d = 0;
    double lat = 0;
    CHECK(s.poll(t, &d, &lat) == kOK && d == 1);
    CHECK(covered[t] == 5);
    CHECK(lat >= prev);
    prev = lat;
  }
  for (auto& L : b.log) {
    int64_t n = 0;
    for (auto& pc : L.pieces) n += pc.count;
    CHECK(n <= 8);
  }
  std::printf("fifo_order ok: %zu launches\n", b.log.size());
}

// A big frame is split over launches; a small one arriving while it renders joins the next
// launch and completes long before the big one.
static void continuous_batching() {
  FakeBackend b;
  Params p;
  p.max_tiles = 100;
  p.max_inflight = 2;
  Sched s(b, p);
  auto tk = drive(s, b, {arrival(0.0, 1000, 0), arrival(50e-6, 3, 1)});
  int d = 0;
  double lat_big = 0, lat_small = 0;
  CHECK(s.poll(tk[0], &d, &lat_big) == kOK && d);
  CHECK(s.poll(tk[1], &d, &lat_small) == kOK && d);
  CHECK(lat_small < 0.5 * lat_big);
  bool shared = false;
  for (auto& L : b.log) shared |= L.pieces.size() == 2;
  CHECK(shared);  // the small frame rode in a launch with part of the big one
  CHECK(b.peak_in_flight <= 2);
  std::printf("continuous_batching ok: big %.1f us, small %.1f us\n", lat_big * 1e6, lat_small * 1e6);
}

// Library images inside a budget of two: the third frame waits until a client frees an
// image; all complete; never more than two images exist.
static void admission_by_budget() {
  FakeBackend b;
  b.budget = 2 * 1000;
  Sched s(b, Params{});
  std::vector<Arrival> arr;
  for (int i = 0; i < 6; ++i) arr.push_back(arrival(0.0, 4, i, &g_group_a, true, 1000));
  std::vector<uint64_t> freed;
  std::vector<uint64_t>* tks = nullptr;
  std::vector<uint64_t> all;
  auto tick = [&]() {
    if (!tks) return;
    for (uint64_t t : *tks) {
      if (!t || std::find(freed.begin(), freed.end(), t) != freed.end()) continue;
      int d = 0;
      if (s.poll(t, &d, nullptr) == kOK && d) {
        float* img = nullptr;
        CHECK(s.image(t, &img) == kOK && img);
        CHECK(s.release(t) == kOK);
        freed.push_back(t);
      }
    }
  };
  // submit first (tickets are known after the first drive step), then free as they finish
  tks = &all;
  all = drive(s, b, arr, [&]() {
    if (all.empty()) {
      for (uint64_t t = 1; t <= 6; ++t) all.push_back(t);
    }
    tick();
  });
  CHECK(freed.size() == 6);
  CHECK(b.peak_used <= 2 * 1000);
  CHECK(b.used == 2 * 1000);  // two images stay pooled for reuse
  CHECK(s.images_held() == 0);
  std::printf("admission_by_budget ok: peak %zu bytes\n", b.peak_used);
}

// The host queue holds at most max_queue frames that are not yet admitted: the next submit
// is refused with kEAGAIN (nothing is admitted while no image fits).
static void eagain_when_queue_full() {
  FakeBackend b;
  b.budget = 0;  // no library image can be allocated
  Params p;
  p.max_queue = 3;
  Sched s(b, p);
  uint64_t t0 = 0, tk = 0;
  CHECK(s.submit(Frame{4, 0}, &g_group_a, nullptr, 1000, &t0) == kOK);
  CHECK(s.submit(Frame{4, 1}, &g_group_a, nullptr, 1000, &tk) == kOK);
  CHECK(s.submit(Frame{4, 2}, &g_group_a, nullptr, 1000, &tk) == kOK);
  CHECK(s.submit(Frame{4, 3}, &g_group_a, nullptr, 1000, &tk) == kEAGAIN);
  // nothing holds an image and nothing is pooled: the queued frames can never fit
  Next n = s.step();
  CHECK(n == Next::kIdle);
  int d = 0;
  CHECK(s.poll(t0, &d, nullptr) == kENOMEM && d == 1);
  CHECK(s.pending() == 0);
  CHECK(s.submit(Frame{4, 4}, &g_group_a, (float*)0x5000, 1000, &tk) == kOK);  // room again
  CHECK(s.step() == Next::kAgain);  // admitted (caller's image) and launched
  s.stop();
  for (int guard = 0; s.step() != Next::kStop; ++guard) {
    CHECK(guard < 10);
    b.t = b.next_end();
  }
  CHECK(s.poll(tk, &d, nullptr) == kOK && d == 1);
  std::printf("eagain_when_queue_full ok\n");
}

// A scripted launch failure fails exactly the frames with tiles in that launch (kEDEVICE);
// frames in the launches before and after it complete normally.
static void launch_failure_is_contained() {
  FakeBackend b;
  b.fail.insert(1);
  Params p;
  p.max_tiles = 10;
  Sched s(b, p);
  // frames over several launches; the second launch fails
  std::vector<Arrival> arr = {arrival(0.0, 10, 0), arrival(0.0, 15, 1), arrival(0.0, 10, 2),
                              arrival(1e-3, 10, 3), arrival(1e-3, 4, 4)};
  auto tk = drive(s, b, arr);
  CHECK(b.log.size() >= 4);
  std::set<uint64_t> in_failed;
  for (auto& pc : b.log[1].pieces) in_failed.insert(pc.ticket);
  CHECK(!in_failed.empty() && in_failed.size() < tk.size());
  for (size_t i = 0; i < tk.size(); ++i) {
    int d = 0;
    int st = s.poll(tk[i], &d, nullptr);
    CHECK(d == 1);
    CHECK(st == (in_failed.count(tk[i]) ? kEDEVICE : kOK));
  }
  // the failed frame's remaining tiles were not launched
  for (size_t k = 2; k < b.log.size(); ++k)
    for (auto& pc : b.log[k].pieces) CHECK(in_failed.count(pc.ticket) == 0);
  std::printf("launch_failure_is_contained ok: %zu failed frames\n", in_failed.size());
}

// Stopping cancels the frames still queued (kECANCELED); admitted frames finish (kOK).
static void cancel_on_stop() {
  FakeBackend b;
  b.budget = 1000;  // one library image at a time
  Sched s(b, Params{});
  std::vector<Arrival> arr;
  for (int i = 0; i < 4; ++i) arr.push_back(arrival(0.0, 20, i, &g_group_a, true, 1000));
  auto tk = drive(s, b, arr, nullptr, 5e-6);  // stop while the first frame renders
  int d = 0;
  CHECK(s.poll(tk[0], &d, nullptr) == kOK && d == 1);
  for (size_t i = 1; i < tk.size(); ++i) CHECK(s.poll(tk[i], &d, nullptr) == kECANCELED && d == 1);
  CHECK(s.pending() == 0);
  uint64_t late = 0;
  CHECK(s.submit(Frame{1, 9}, &g_group_a, nullptr, 10, &late) == kEINVAL);
  std::printf("cancel_on_stop ok\n");
}

// Frames of different table sets never share a launch; at most max_inflight launches are
// in flight.
static void one_table_set_per_launch() {
  FakeBackend b;
  Params p;
  p.max_inflight = 3;
  Sched s(b, p);
  std::vector<Arrival> arr;
  for (int i = 0; i < 12; ++i) arr.push_back(arrival(i * 2e-6, 3, i, i % 3 ? &g_group_a : &g_group_b));
  auto tk = drive(s, b, arr);
  for (auto& L : b.log)
    for (auto& pc : L.pieces) {
      const void* g = arr[pc.ticket - 1].group;
      CHECK(g == L.group);
    }
  CHECK(b.peak_in_flight <= 3);
  for (uint64_t t : tk) {
    int d = 0;
    CHECK(s.poll(t, &d, nullptr) == kOK && d == 1);
  }
  std::printf("one_table_set_per_launch ok: %zu launches\n", b.log.size());
}

// Releasing pooled images makes room for a larger one: freed images of another size are
// given back to the backend (largest first) when a new size does not fit.
static void pool_gives_back_for_other_sizes() {
  FakeBackend b;
  b.budget = 3000;
  Sched s(b, Params{});
  std::vector<uint64_t> tks;
  auto free_done = [&]() {
    for (uint64_t t : tks) {
      int d = 0;
      if (t && s.poll(t, &d, nullptr) == kOK && d) (void)s.release(t);
    }
  };
  std::vector<Arrival> arr = {arrival(0.0, 2, 0, &g_group_a, true, 1000),
                              arrival(0.0, 2, 1, &g_group_a, true, 1000),
                              arrival(1e-3, 2, 2, &g_group_a, true, 2500)};
  tks = drive(s, b, arr, [&]() {
    if (tks.empty()) tks = {1, 2, 3};
    free_done();
  });
  int d = 0;
  CHECK(s.poll(3, &d, nullptr) == kENOTFOUND);  // all three finished and were freed
  CHECK(b.used == 2500);                        // the two small images went back
  std::printf("pool_gives_back_for_other_sizes ok\n");
}

// ---- real-time backend and threads (for TSan) ------------------------------------------------
struct RealBackend {
  using Payload = Frame;
  struct Handle {
    int64_t id = -1;
  };
  using clock = std::chrono::steady_clock;
  clock::time_point t0 = clock::now();
  double stream_free = 0;
  std::map<int64_t, double> end;  // scheduler thread only
  int64_t next_id = 0;
  std::atomic<int64_t> launches{0};
  size_t budget = 64 * 1000, used = 0;
  uintptr_t next_addr = 0x10000;
  std::map<uintptr_t, size_t> live;

  double now() { return std::chrono::duration<double>(clock::now() - t0).count(); }
  int64_t tiles(const Frame& f) { return f.tiles; }
  void* try_alloc(size_t bytes) {
    if (used + bytes > budget) return nullptr;
    used += bytes;
    uintptr_t a = next_addr;
    next_addr += 0x1000;
    live[a] = bytes;
    return (void*)a;
  }
  void dealloc(void* p, size_t bytes) {
    CHECK(live.erase((uintptr_t)p) == 1);
    used -= bytes;
  }
  int launch(const std::vector<Piece<Frame>>&, int64_t ntiles, Handle* h) {
    h->id = next_id++;
    const double start = std::max(now(), stream_free);
    end[h->id] = stream_free = start + 20e-6 + 1e-6 * (double)ntiles;
    launches++;
    return kOK;
  }
  bool done(Handle& h) { return now() >= end.at(h.id); }
  void wait(Handle& h) {
    while (!done(h)) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  void release(Handle& h) { end.erase(h.id); }
};

// Four client threads submit, poll and free frames while the scheduler thread runs; then
// drain, stop and join.  Every frame completes with kOK and every image is given back.
static void threads() {
  RealBackend b;
  Params p;
  p.max_tiles = 64;
  p.max_queue = 1000;
  auto* s = new Scheduler<RealBackend>(b, p);
  std::thread sched([s] { s->run(); });
  std::atomic<int> ok{0};
  std::vector<std::thread> clients;
  for (int c = 0; c < 4; ++c)
    clients.emplace_back([&, c] {
      std::vector<uint64_t> mine;
      for (int i = 0; i < 60; ++i) {
        uint64_t tk = 0;
        int rc;
        while ((rc = s->submit(Frame{1 + (i * 7 + c) % 50, i}, c % 2 ? &g_group_a : &g_group_b,
                               nullptr, 1000, &tk)) == kEAGAIN)
          std::this_thread::yield();
        CHECK(rc == kOK);
        mine.push_back(tk);
        // keep at most 8 frames of this client alive: free the finished ones
        while (mine.size() > 8) {
          int d = 0;
          int st = s->poll(mine.front(), &d, nullptr);
          if (!d) {
            std::this_thread::sleep_for(std::chrono::microseconds(50));
            continue;
          }
          CHECK(st == kOK);
          ok++;
          CHECK(s->release(mine.front()) == kOK);
          mine.erase(mine.begin());
        }
      }
      for (uint64_t tk : mine) {
        int d = 0;
        while (s->poll(tk, &d, nullptr) == kOK && !d) std::this_thread::sleep_for(std::chrono::microseconds(50));
        ok++;
        CHECK(s->release(tk) == kOK);
      }
    });
  for (auto& t : clients) t.join();
  s->drain();
  s->stop();
  sched.join();
  CHECK(ok.load() == 240);
  delete s;
  CHECK(b.used == 0 && b.live.empty());
  std::printf("threads ok: %lld launches\n", (long long)b.launches.load());
}

int main(int argc, char** argv) {
  const std::string which = argc > 1 ? argv[1] : "all";
  const std::vector<std::pair<std::string, void (*)()>> all = {
      {"fifo_order", fifo_order},
      {"continuous_batching", continuous_batching},
      {"admission_by_budget", admission_by_budget},
      {"eagain_when_queue_full", eagain_when_queue_full},
      {"launch_failure_is_contained", launch_failure_is_contained},
      {"cancel_on_stop", cancel_on_stop},
      {"one_table_set_per_launch", one_table_set_per_launch},
      {"pool_gives_back_for_other_sizes", pool_gives_back_for_other_sizes},
      {"threads", threads},
  };
  bool found = false;
  for (auto& kv : all)
    if (which == "all" || which == kv.first) {
      kv.second();
      found = true;
    }
  if (!found) {
    std::fprintf(stderr, "unknown scenario %s\n", which.c_str());
    return 2;
  }
  return 0;
}
