// Host-side bookkeeping of the continuous-batching server: carving of the
// device pool, admission order and the life of every request.  It makes no
// HIP call: the server drives it under its mutex and performs the device work
// (stream waits, sketch launches, completion markers) itself, and a CPU test
// drives it with simulated completions.
//
// Life of a request:
//   QUEUED     submitted, waiting for a slot and pool space
//   LAUNCHING  admitted: owns a slot and a pool range; its kernels are being
//              enqueued on the slot's stream (outside the server mutex)
//   RUNNING    enqueued, completion marker placed behind its last kernel
//   DONE       the marker has fired; pool range and slot are free again
//   FAILED     as DONE, but the launch sequence stopped on an error.  Kernels
//              enqueued before the error may still have been running, so the
//              pool range is held until the marker behind them has fired.
//   CANCELED   removed while QUEUED
//
// Admission: requests are considered in arrival order; one that does not fit
// the pool (or finds no free slot) may be passed by later ones, but only
// max_bypass times: after that nothing behind it is admitted until it fits,
// so a large request cannot starve.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <map>
#include <vector>

namespace cabs_serve {

struct Block {
  size_t off, size;
};

// First-fit allocator over [0, capacity) in 256-byte units, with coalescing of
// free neighbours.
class Pool {
 public:
  explicit Pool(size_t cap) : cap_(cap) {
    if (cap) free_.push_back({0, cap});
  }
  static size_t round(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
  bool alloc(size_t bytes, size_t& off) {
    bytes = round(bytes);
    for (size_t i = 0; i < free_.size(); ++i) {
      if (free_[i].size >= bytes) {
        off = free_[i].off;
        free_[i].off += bytes;
        free_[i].size -= bytes;
        if (free_[i].size == 0) free_.erase(free_.begin() + i);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round(bytes);
    size_t i = 0;
    while (i < free_.size() && free_[i].off < off) ++i;
    free_.insert(free_.begin() + i, {off, bytes});
    if (i + 1 < free_.size() && free_[i].off + free_[i].size == free_[i + 1].off) {
      free_[i].size += free_[i + 1].size;
      free_.erase(free_.begin() + i + 1);
    }
    if (i > 0 && free_[i - 1].off + free_[i - 1].size == free_[i].off) {
      free_[i - 1].size += free_[i].size;
      free_.erase(free_.begin() + i);
    }
  }
  size_t capacity() const { return cap_; }
  size_t free_bytes() const {
    size_t s = 0;
    for (const Block& b : free_) s += b.size;
    return s;
  }
  size_t free_ranges() const { return free_.size(); }

 private:
  size_t cap_;
  std::vector<Block> free_;
};

enum State { QUEUED = 0, LAUNCHING, RUNNING, DONE, FAILED, CANCELED };

struct Entry {
  uint64_t ticket = 0;
  size_t bytes = 0;
  size_t off = 0;
  int slot = -1;
  State state = QUEUED;
  int status = 0;   // error of a FAILED request
  int passed = 0;   // times a later request was admitted while this one waited
};

struct Launch {
  uint64_t ticket;
  int slot;
  size_t off;
  size_t bytes;
};

class Core {
 public:
  Core(size_t capacity, int slots, int max_bypass)
      : pool_(capacity), slot_(slots, 0), max_bypass_(max_bypass) {}

  // A new QUEUED request needing `bytes` of pool; 0 if it can never fit.
  uint64_t submit(size_t bytes) {
    if (Pool::round(bytes) > pool_.capacity()) return 0;
    Entry e;
    e.ticket = next_++;
    e.bytes = bytes;
    reqs_[e.ticket] = e;
    queue_.push_back(e.ticket);
    return e.ticket;
  }

  // Admissions for this round (see the file comment).  Admitted requests are
  // LAUNCHING and own their slot and pool range.
  std::vector<Launch> admit() {
    std::vector<Launch> out;
    std::vector<uint64_t> waiting;  // considered and not admitted, in order
    for (auto it = queue_.begin(); it != queue_.end();) {
      int slot = -1;
      for (size_t k = 0; k < slot_.size(); ++k)
        if (!slot_[k]) { slot = (int)k; break; }
      if (slot < 0) break;
      Entry& e = reqs_[*it];
      size_t off = 0;
      if (!pool_.alloc(e.bytes, off)) {
        waiting.push_back(e.ticket);
        if (e.passed >= max_bypass_) break;  // nothing may pass it any more
        ++it;
        continue;
      }
      for (uint64_t w : waiting) ++reqs_[w].passed;
      e.state = LAUNCHING;
      e.slot = slot;
      e.off = off;
      slot_[slot] = e.ticket;
      ++running_;
      out.push_back({e.ticket, slot, off, e.bytes});
      it = queue_.erase(it);
    }
    return out;
  }

  // The launch sequence of a LAUNCHING request has ended.  marker = true: the
  // slot's completion marker was placed behind whatever was enqueued, and the
  // request is RUNNING until retire() sees it fire (status != 0 makes it end
  // FAILED).  marker = false: the caller has waited for the slot's stream
  // itself, so the request ends at once (FAILED with status).
  void launched(uint64_t ticket, int status, bool marker) {
    Entry& e = reqs_[ticket];
    e.status = status;
    e.state = RUNNING;
    if (!marker) finish(e);
  }

  // Retire every RUNNING request whose slot marker `done(slot)` reports as
  // fired; returns their tickets.
  template <class F>
  std::vector<uint64_t> retire(F done) {
    std::vector<uint64_t> out;
    for (size_t k = 0; k < slot_.size(); ++k) {
      const uint64_t t = slot_[k];
      if (!t) continue;
      Entry& e = reqs_[t];
      if (e.state != RUNNING || !done((int)k)) continue;
      finish(e);
      out.push_back(t);
    }
    return out;
  }

  // Cancel a QUEUED request: 0 done, 1 already admitted, -1 unknown ticket.
  int cancel(uint64_t ticket) {
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return -1;
    if (it->second.state != QUEUED) return it->second.state == DONE || it->second.state == FAILED ||
                                                   it->second.state == CANCELED
                                               ? 0
                                               : 1;
    for (auto q = queue_.begin(); q != queue_.end(); ++q)
      if (*q == ticket) { queue_.erase(q); break; }
    it->second.state = CANCELED;
    return 0;
  }

  const Entry* find(uint64_t ticket) const {
    auto it = reqs_.find(ticket);
    return it == reqs_.end() ? nullptr : &it->second;
  }
  void forget(uint64_t ticket) { reqs_.erase(ticket); }

  bool idle() const { return queue_.empty() && running_ == 0; }
  int running() const { return running_; }
  size_t queued() const { return queue_.size(); }
  const Pool& pool() const { return pool_; }

 private:
  void finish(Entry& e) {
    e.state = e.status ? FAILED : DONE;
    pool_.release(e.off, e.bytes);
    slot_[e.slot] = 0;
    --running_;
  }

  Pool pool_;
  std::vector<uint64_t> slot_;
  std::deque<uint64_t> queue_;
  std::map<uint64_t, Entry> reqs_;
  uint64_t next_ = 1;
  int running_ = 0;
  int max_bypass_;
};

}  // namespace cabs_serve
