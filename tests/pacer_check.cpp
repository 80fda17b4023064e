// Host check of the solve pacing (csrc/pacer.h) against a simulated device
// that runs queued chunks in order. Prints the first violated property and
// exits non-zero.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "pacer.h"

using fi::kAhead;
using fi::kPredMargin;

static int g_fail = 0;
#define CHECK(c, ...)                                    \
  do {                                                   \
    if (!(c)) {                                          \
      std::printf("FAIL %s: ", #c);                      \
      std::printf(__VA_ARGS__);                          \
      std::printf("\n");                                 \
      g_fail = 1;                                        \
      return -1;                                         \
    }                                                    \
  } while (0)

static int kChunk = fi::kChunk;  // the chunk of the pacers under test

// A solve that needs `end` step launches. The host sees its end once the
// chunk holding launch `end` has run. Returns the launches queued by then,
// or -2 when the host stops at the limit without seeing the end.
static long long run(long long max_inner, long long max_refine, long long pred, long long end) {
  fi::Pacer p = fi::make_pacer(max_inner, max_refine, pred, kChunk);
  CHECK(p.chunk == kChunk, "chunk %d, asked for %d", p.chunk, kChunk);
  std::vector<int> chunks;
  long long executed = 0;
  for (long long step = 0; step < 10000000; ++step) {
    if (executed >= end) return p.queued;
    const int n = p.next();
    if (n) {
      CHECK(n % 2 == 0 && n >= 2 && n <= kChunk, "chunk of %d launches", n);
      CHECK(p.queued + n <= p.limit, "queued %lld + %d past the limit %lld", (long long)p.queued, n,
            (long long)p.limit);
      chunks.push_back(n);
      p.queued_chunk(n);
      CHECK(p.launched - p.completed <= kAhead, "%lld chunks in flight",
            (long long)(p.launched - p.completed));
      continue;
    }
    if (p.completed < p.launched) {
      executed += chunks[p.completed];
      ++p.completed;
      continue;
    }
    CHECK(p.queued >= p.limit, "stalled at %lld queued (limit %lld) with nothing in flight",
          (long long)p.queued, (long long)p.limit);
    return -2;
  }
  CHECK(false, "no progress");
  return -1;
}

static int check_all() {
  const long long mi = 20000, mr = 40;
  for (long long end = 1; end <= 400 && !g_fail; ++end) {
    // no prediction: at most the chunks in flight run idle
    long long q = run(mi, mr, 0, end);
    CHECK(q >= end && q - end < (kAhead + 1) * kChunk, "no prediction: end %lld queued %lld", end, q);
    // an exact or long prediction stops near it
    for (long long over : {0LL, 1LL, 3LL, 17LL, 200LL}) {
      q = run(mi, mr, end + over, end);
      CHECK(q >= end && q <= end + over + kPredMargin + 1,
            "prediction %lld: end %lld queued %lld", end + over, end, q);
    }
    // a short prediction still reaches the end, one drain later
    for (long long under : {1LL, 2LL, 9LL, 50LL}) {
      if (under >= end) continue;
      q = run(mi, mr, end - under, end);
      CHECK(q >= end && q - end < (kAhead + 1) * kChunk, "prediction %lld: end %lld queued %lld",
            end - under, end, q);
    }
  }
  // tight caps: the host never queues past the limit, and reports a solve
  // that needs more as not ended
  for (long long end = 1; end <= 80 && !g_fail; ++end) {
    for (long long pred : {0LL, 5LL, 31LL, 500LL}) {
      fi::Pacer p = fi::make_pacer(1, 1, pred, kChunk);
      const long long q = run(1, 1, pred, end);
      if (end <= p.limit) {
        CHECK(q >= end && q <= p.limit, "cap: end %lld pred %lld queued %lld", end, pred, q);
      } else {
        CHECK(q == -2, "cap: end %lld past the limit %lld, got %lld", end, (long long)p.limit, q);
      }
    }
  }
  return 0;
}

int main() {
  for (int c : {fi::kChunk, fi::kChunkShort, 2, 6}) {
    kChunk = c;
    check_all();
    if (g_fail) {
      std::printf("(chunks of %d)\n", c);
      return 1;
    }
  }
  if (fi::make_pacer(10, 1, 0, 7).chunk != 6 || fi::make_pacer(10, 1, 0, 1).chunk != 2) {
    std::printf("FAIL: odd chunk sizes are not rounded down to even\n");
    return 1;
  }
  if (fi::launches_used(86, 3) != 93) {
    std::printf("FAIL: launch count\n");
    return 1;
  }
  std::printf("pacer: all properties hold\n");
  return 0;
}
