// CPU checks of the server's bookkeeping (serve_core.hpp) with simulated
// completions: pool carving and coalescing, admission with bounded bypass,
// workspace held by a failed request until its completion marker fires,
// cancellation.  Prints one line per check; exit status 0 when all hold.
#include <cstdio>
#include <cstdlib>
#include <set>

#include "serve_core.hpp"

using namespace cabs_serve;

static int g_fail = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #cond);      \
      ++g_fail;                                                       \
    }                                                                 \
  } while (0)

static void pool_checks() {
  Pool p(1 << 20);
  size_t a, b, c;
  CHECK(p.alloc(1000, a) && a == 0);
  CHECK(p.alloc(300, b) && b == 1024);
  CHECK(p.alloc(1, c) && c == 1024 + 512);
  p.release(b, 300);
  CHECK(p.free_ranges() == 2);
  p.release(a, 1000);  // coalesces with the hole left by b
  CHECK(p.free_ranges() == 2);
  p.release(c, 1);     // everything free again: one range
  CHECK(p.free_ranges() == 1 && p.free_bytes() == (1u << 20));
  size_t x;
  CHECK(!p.alloc((1 << 20) + 1, x));
  // random churn keeps the free list consistent: allocations never overlap
  std::srand(7);
  std::set<std::pair<size_t, size_t>> live;
  for (int it = 0; it < 20000; ++it) {
    if (!live.empty() && (std::rand() & 1)) {
      auto i = live.begin();
      std::advance(i, std::rand() % live.size());
      p.release(i->first, i->second);
      live.erase(i);
    } else {
      size_t sz = 1 + std::rand() % 50000, off;
      if (p.alloc(sz, off)) {
        const size_t r = Pool::round(sz);
        for (auto& q : live) CHECK(off + r <= q.first || Pool::round(q.second) + q.first <= off);
        live.insert({off, sz});
      }
    }
  }
  for (auto& q : live) p.release(q.first, q.second);
  CHECK(p.free_ranges() == 1 && p.free_bytes() == (1u << 20));
  std::printf("pool ok\n");
}

static void bypass_checks() {
  // 2 slots, pool of 10 units of 256 B; max_bypass 2
  Core c(10 * 256, 2, 2);
  const uint64_t big = c.submit(8 * 256);
  const uint64_t big2 = c.submit(8 * 256);  // waits for big
  auto adm = c.admit();
  CHECK(adm.size() == 1 && adm[0].ticket == big);
  c.launched(big, 0, true);
  // small requests pass the waiting big2 at most twice
  const uint64_t s1 = c.submit(256), s2 = c.submit(256), s3 = c.submit(256);
  adm = c.admit();
  CHECK(adm.size() == 1 && adm[0].ticket == s1);  // one free slot
  c.launched(s1, 0, true);
  auto ret = c.retire([&](int slot) { return slot == adm[0].slot; });
  CHECK(ret.size() == 1 && ret[0] == s1);
  adm = c.admit();
  CHECK(adm.size() == 1 && adm[0].ticket == s2);
  c.launched(s2, 0, true);
  ret = c.retire([&](int slot) { return slot == adm[0].slot; });
  CHECK(ret.size() == 1);
  CHECK(c.find(big2)->passed == 2);
  adm = c.admit();  // big2 has been passed twice: s3 must wait behind it
  CHECK(adm.empty());
  // big finishes; big2 fits, then s3 runs beside it
  ret = c.retire([&](int) { return true; });
  CHECK(ret.size() == 1 && ret[0] == big);
  adm = c.admit();
  CHECK(adm.size() == 2 && adm[0].ticket == big2 && adm[1].ticket == s3);
  for (auto& a : adm) c.launched(a.ticket, 0, true);
  ret = c.retire([&](int) { return true; });
  CHECK(ret.size() == 2 && c.idle());
  CHECK(c.find(s3)->state == DONE);
  std::printf("bypass ok\n");
}

static void failed_launch_checks() {
  // a launch that fails after enqueuing kernels keeps its workspace until the marker fires
  Core c(4 * 256, 2, 8);
  const uint64_t a = c.submit(4 * 256);
  auto adm = c.admit();
  CHECK(adm.size() == 1);
  c.launched(a, -4, true);
  CHECK(c.find(a)->state == RUNNING);
  const uint64_t b = c.submit(4 * 256);
  CHECK(c.admit().empty());  // a's range is still reserved
  auto ret = c.retire([](int) { return false; });
  CHECK(ret.empty() && c.admit().empty());
  ret = c.retire([](int) { return true; });
  CHECK(ret.size() == 1 && c.find(a)->state == FAILED && c.find(a)->status == -4);
  adm = c.admit();
  CHECK(adm.size() == 1 && adm[0].ticket == b && adm[0].off == 0);
  // no marker could be placed (the caller synchronised the stream): ends at once
  c.launched(b, -4, false);
  CHECK(c.find(b)->state == FAILED && c.idle());
  std::printf("failed launch ok\n");
}

static void cancel_checks() {
  Core c(4 * 256, 1, 8);
  const uint64_t a = c.submit(256), b = c.submit(256);
  CHECK(c.cancel(b) == 0 && c.find(b)->state == CANCELED);
  auto adm = c.admit();
  CHECK(adm.size() == 1 && adm[0].ticket == a);
  CHECK(c.cancel(a) == 1);  // already admitted
  c.launched(a, 0, true);
  c.retire([](int) { return true; });
  CHECK(c.idle() && c.cancel(12345) == -1);
  CHECK(c.submit(5 * 256) == 0);  // can never fit
  std::printf("cancel ok\n");
}

int main() {
  pool_checks();
  bypass_checks();
  failed_launch_checks();
  cancel_checks();
  std::printf(g_fail ? "FAILED %d\n" : "all ok\n", g_fail);
  return g_fail ? 1 : 0;
}
