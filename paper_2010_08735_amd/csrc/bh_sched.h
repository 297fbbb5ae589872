// Serving scheduler of libbh: continuous batching of frame requests.  Plain C++17, no HIP:
// the device side is a Backend (the HIP one in libbh.cpp; a scripted one with a virtual
// clock in the CPU tests), so the whole policy runs and is tested without a GPU.
//
// Policy.  Requests are admitted in arrival order while their images fit: a request
// without a caller image gets one from the pool of freed images of the same size, else a
// new one from the backend inside its memory budget, releasing pooled images (largest
// first) if that is what it takes; if nothing fits and no image is held by a request, it
// never will, and the request fails with kENOMEM.  Each step fills one launch with up to
// max_tiles tiles from the admitted requests of one table set (group): the oldest admitted
// request is guaranteed up to half of the launch, the other requests of its group follow in
// order of fewest remaining tiles (ties by age), and the oldest takes whatever room is
// left.  A frame larger than a launch spills into the next ones while frames that arrive
// meanwhile still join the next launch, and no request waits forever.  At most max_inflight
// launches are in flight; a request completes with the launch that holds its last tile,
// and a failed launch fails every request with tiles in it (the others are untouched).
// Stopping cancels the requests still queued; admitted ones run to completion.
//
// Threads.  Client calls (submit, poll, image, release, drain, stop) may come from any
// thread.  step() runs on one scheduler thread and never blocks; run() is that thread's
// loop and does the waiting step() asks for.  Everything shared lives under mu_.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <utility>
#include <vector>

namespace bh {
namespace sched {

// status codes, numerically those of bh_status
enum Status : int {
  kOK = 0, kEINVAL = 1, kENOMEM = 2, kEDEVICE = 3, kEAGAIN = 4, kENOTFOUND = 5, kECANCELED = 6
};

struct Params {
  int max_queue = 1 << 20;     // submitted but not yet admitted
  int max_inflight = 6;        // launches in flight
  int64_t max_tiles = 262144;  // tiles per launch
};

template <class Payload>
struct Request {
  uint64_t ticket = 0;
  Payload payload{};           // what the backend renders (view record, tables, ...)
  const void* group = nullptr; // requests of one launch share it (their table set)
  float* out = nullptr;        // image (caller's, or the library's once admitted)
  bool owned = false;          // out belongs to the library
  size_t out_bytes = 0;
  int64_t tiles_total = -1, tiles_next = 0;  // scheduler thread only
  double t_submit = 0, t_done = 0;
  bool admitted = false, done = false;
  int status = kOK;
};

// tiles [first, first + count) of request r go into a launch
template <class Payload>
struct Piece {
  Request<Payload>* r;
  int64_t first, count;
};

// What the scheduler thread should wait for after a step.
enum class Next { kStop, kIdle, kPoll, kWaitOldest, kAgain };

// Backend requirements (B):
//   using Payload; using Handle;                     a launch in flight
//   double now();
//   int64_t tiles(const Payload&);                   tiles of the frame (current tile shape)
//   void* try_alloc(size_t bytes);                   inside the budget, or nullptr
//   void dealloc(void* p, size_t bytes);
//   int launch(const std::vector<Piece<Payload>>&, int64_t ntiles, Handle* h);
//        enqueues the launch; *h is valid (it completes after every earlier launch) even
//        when the status is not kOK, in which case no tile of it is rendered
//   bool done(Handle&);  void wait(Handle&);  void release(Handle&);
template <class B>
class Scheduler {
 public:
  using Payload = typename B::Payload;
  using Req = Request<Payload>;

  Scheduler(B& backend, const Params& p) : b_(backend), p_(p) {
    p_.max_queue = std::max(1, p_.max_queue);
    p_.max_inflight = std::max(1, p_.max_inflight);
    p_.max_tiles = std::max<int64_t>(1, p_.max_tiles);
  }
  Scheduler(const Scheduler&) = delete;
  Scheduler& operator=(const Scheduler&) = delete;

  // Frees every request and pooled image; call after the scheduler thread has ended.
  ~Scheduler() {
    for (auto& kv : reqs_) {
      if (kv.second->owned) b_.dealloc(kv.second->out, kv.second->out_bytes);
      delete kv.second;
    }
    for (auto& kv : pool_) b_.dealloc(kv.second, kv.first);
  }

  // ---- client side ------------------------------------------------------------------------

  // out == nullptr: the library allocates the image (out_bytes) at admission
  int submit(const Payload& pl, const void* group, float* out, size_t out_bytes,
             uint64_t* ticket) {
    std::lock_guard<std::mutex> g(mu_);
    if (stop_) return kEINVAL;
    if ((int)queue_.size() >= p_.max_queue) return kEAGAIN;
    auto* r = new Req;
    r->ticket = next_ticket_++;
    r->payload = pl;
    r->group = group;
    r->out = out;
    r->out_bytes = out_bytes;
    r->t_submit = b_.now();
    reqs_[r->ticket] = r;
    queue_.push_back(r);
    pending_++;
    *ticket = r->ticket;
    cv_.notify_all();
    return kOK;
  }

  // done = 1 once the frame is complete (or failed); the request's status is returned
  int poll(uint64_t ticket, int* done, double* latency) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return kENOTFOUND;
    Req* r = it->second;
    *done = r->done ? 1 : 0;
    if (latency) *latency = (r->done ? r->t_done : b_.now()) - r->t_submit;
    return r->status;
  }

  int image(uint64_t ticket, float** img) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return kENOTFOUND;
    if (!it->second->done) return kEAGAIN;
    *img = it->second->out;
    return kOK;
  }

  // forget a finished request; its library image goes back to the pool
  int release(uint64_t ticket) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return kENOTFOUND;
    if (!it->second->done) return kEAGAIN;
    if (it->second->owned) {
      pool_.emplace(it->second->out_bytes, it->second->out);
      owned_live_--;
    }
    delete it->second;
    reqs_.erase(it);
    cv_.notify_all();  // a freed image may admit queued requests
    return kOK;
  }

  void drain() {
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return pending_ == 0; });
  }

  // Cancel the queued requests and let the scheduler finish what it has admitted; run()
  // returns (step() answers kStop) once nothing is left in flight.
  void stop() {
    std::lock_guard<std::mutex> g(mu_);
    for (Req* r : queue_) finish(r, kECANCELED, b_.now());
    queue_.clear();
    stop_ = true;
    cv_.notify_all();
  }

  size_t pending() {
    std::lock_guard<std::mutex> g(mu_);
    return pending_;
  }
  int64_t images_held() {
    std::lock_guard<std::mutex> g(mu_);
    return owned_live_;
  }
  size_t inflight() const { return inflight_.size(); }  // scheduler thread

  // ---- scheduler side ---------------------------------------------------------------------

  // One iteration; never blocks.  The answer says what to wait for before the next one.
  Next step() {
    // retire the launches that have finished, in order
    while (!inflight_.empty() && b_.done(inflight_.front().h)) {
      Flight& f = inflight_.front();
      const double t = b_.now();
      {
        std::lock_guard<std::mutex> g(mu_);
        for (uint64_t tk : f.finishing) {
          auto it = reqs_.find(tk);
          if (it != reqs_.end() && !it->second->done) finish(it->second, it->second->status, t);
        }
      }
      b_.release(f.h);
      inflight_.pop_front();
    }
    {
      std::lock_guard<std::mutex> g(mu_);
      admit();
      if (stop_ && queue_.empty() && active_.empty() && inflight_.empty()) return Next::kStop;
      if (active_.empty()) return inflight_.empty() ? Next::kIdle : Next::kPoll;
    }
    if ((int)inflight_.size() >= p_.max_inflight) return Next::kWaitOldest;
    fill_and_launch();
    return Next::kAgain;
  }

  // Block until the oldest launch in flight has finished (what kWaitOldest asks for).
  void wait_oldest() {
    if (!inflight_.empty()) b_.wait(inflight_.front().h);
  }

  // The scheduler thread: step, then wait as asked.
  void run() {
    using namespace std::chrono;
    for (;;) {
      const Next n = step();
      if (n == Next::kStop) return;
      if (n == Next::kWaitOldest) {
        wait_oldest();
      } else if (n == Next::kIdle || n == Next::kPoll) {
        // idle: wait for a request or a freed image; launches in flight: poll soon.  (A
        // system_clock deadline waits through pthread_cond_timedwait, which thread
        // sanitizers see release the mutex; steady_clock waits use pthread_cond_clockwait.)
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait_until(lk, system_clock::now() +
                               (n == Next::kIdle ? microseconds(2000) : microseconds(50)));
      }
    }
  }

 private:
  struct Flight {
    typename B::Handle h{};
    std::vector<uint64_t> finishing;  // tickets whose last tile is in this launch
  };

  // caller holds mu_
  void finish(Req* r, int status, double t) {
    r->status = status;
    r->done = true;
    r->t_done = t;
    pending_--;
    done_cv_.notify_all();
  }

  // a library image of `bytes`: pooled one of that size, else a new one, releasing pooled
  // images (largest first) until it fits; caller holds mu_
  void* get_image(size_t bytes) {
    auto it = pool_.find(bytes);
    if (it != pool_.end()) {
      void* p = it->second;
      pool_.erase(it);
      return p;
    }
    for (;;) {
      if (void* p = b_.try_alloc(bytes)) return p;
      if (pool_.empty()) return nullptr;
      auto big = std::prev(pool_.end());
      b_.dealloc(big->second, big->first);
      pool_.erase(big);
    }
  }

  // admission in arrival order; caller holds mu_
  void admit() {
    while (!queue_.empty()) {
      Req* r = queue_.front();
      if (!r->out) {
        void* p = get_image(r->out_bytes);
        if (!p) {
          if (owned_live_ > 0) break;  // wait for a client to free an image
          // nothing held and nothing pooled: this image can never be allocated
          queue_.pop_front();
          finish(r, kENOMEM, b_.now());
          continue;
        }
        r->out = (float*)p;
        r->owned = true;
        owned_live_++;
      }
      r->admitted = true;
      queue_.pop_front();
      active_.push_back(r);
    }
  }

  // one launch from the admitted requests (scheduler thread only)
  void fill_and_launch() {
    Req* oldest = active_.front();
    const void* group = oldest->group;  // one table set per launch
    for (Req* r : active_)
      if (r->tiles_total < 0) r->tiles_total = b_.tiles(r->payload);
    auto left = [](const Req* r) { return r->tiles_total - r->tiles_next; };
    // the oldest keeps up to half of the launch; the others of its group fill the rest,
    // fewest remaining tiles first (stable: ties keep their admission order)
    const int64_t reserve = std::min(left(oldest), (p_.max_tiles + 1) / 2);
    std::vector<Req*> others;
    for (size_t k = 1; k < active_.size(); ++k)
      if (active_[k]->group == group) others.push_back(active_[k]);
    std::stable_sort(others.begin(), others.end(),
                     [&](const Req* a, const Req* b) { return left(a) < left(b); });
    std::vector<std::pair<Req*, int64_t>> takes;  // (request, tiles), the oldest first
    int64_t used = 0;
    for (Req* r : others) {
      const int64_t room = p_.max_tiles - reserve - used;
      if (room <= 0) break;
      const int64_t take = std::min(left(r), room);
      takes.emplace_back(r, take);
      used += take;
    }
    takes.insert(takes.begin(), std::make_pair(oldest, std::min(left(oldest), p_.max_tiles - used)));
    std::vector<Piece<Payload>> pieces;
    Flight f;
    int64_t ntiles = 0;
    for (auto& rt : takes) {
      Req* r = rt.first;
      if (rt.second <= 0) continue;
      pieces.push_back(Piece<Payload>{r, r->tiles_next, rt.second});
      ntiles += rt.second;
      r->tiles_next += rt.second;
      if (r->tiles_next >= r->tiles_total) f.finishing.push_back(r->ticket);
    }
    active_.erase(std::remove_if(active_.begin(), active_.end(),
                                 [](Req* r) { return r->tiles_next >= r->tiles_total; }),
                  active_.end());
    const int st = b_.launch(pieces, ntiles, &f.h);
    if (st != kOK) {
      // every request with tiles in this launch fails; the unfinished ones stop here
      std::lock_guard<std::mutex> g(mu_);
      for (const auto& pc : pieces) {
        Req* r = pc.r;
        r->status = st;
        if (r->tiles_next < r->tiles_total) {
          r->tiles_next = r->tiles_total;
          f.finishing.push_back(r->ticket);
        }
      }
      active_.erase(std::remove_if(active_.begin(), active_.end(),
                                   [](Req* r) { return r->status != kOK; }),
                    active_.end());
    }
    inflight_.push_back(std::move(f));
  }

  B& b_;
  Params p_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::deque<Req*> queue_;                    // submitted, not admitted (under mu_)
  std::unordered_map<uint64_t, Req*> reqs_;   // every live request (under mu_)
  std::multimap<size_t, void*> pool_;         // freed library images by size (under mu_)
  uint64_t next_ticket_ = 1;
  size_t pending_ = 0;                        // submitted, not finished (under mu_)
  int64_t owned_live_ = 0;                    // library images held by requests (under mu_)
  bool stop_ = false;                         // (under mu_)
  std::vector<Req*> active_;                  // admitted, tiles left (scheduler thread)
  std::deque<Flight> inflight_;               // launches in flight (scheduler thread)
};

}  // namespace sched
}  // namespace bh
