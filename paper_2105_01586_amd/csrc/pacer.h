// Host pacing of a solve's step launches (plain C++, no device code).
//
// The host queues step launches in chunks, each followed by an event, keeps
// at most kAhead chunks queued, and stops once the solve reports its end.
// Launches queued past the end run idle (they carry the final record
// forward and change no result), so the host also stops queueing at the
// launch count the previous solve of the same kind took, plus kPredMargin;
// if the solve is still running once all of those have run, pacing goes on
// as without a prediction. Every chunk has an even number of launches, so
// launch k of a solve always has parity k % 2. Short launches (a grid that
// runs in one round) go in longer chunks: fewer events and host wake-ups
// per launch.
#pragma once

#include <algorithm>
#include <cstdint>

namespace fi {

constexpr int kChunk = 8;       // step launches per chunk (even)
constexpr int kChunkShort = 16; // step launches per chunk of short launches (even)
constexpr int kAhead = 2;       // chunks queued at most
constexpr int kPredMargin = 0;  // launches queued beyond the prediction (rounded up to even)

// Step launches a solve used: one per iteration, the start and the end of
// every inner solve, and the launch that found the outer tolerance met.
inline int64_t launches_used(int64_t iterations, int64_t inner_solves) {
  return iterations + 2 * inner_solves + 1;
}

struct Pacer {
  int64_t cap;    // launches to queue before waiting for the end
  int64_t limit;  // launches never exceeded
  int chunk = kChunk;  // launches per chunk (even)
  int64_t queued = 0, launched = 0, completed = 0;  // launches; chunks; chunks
  // Launches to queue now as one chunk (even), or 0 to wait.
  int next() {
    if (launched - completed >= kAhead || queued >= limit) return 0;
    if (queued >= cap) {
      if (completed != launched) return 0;
      cap = limit;  // the prediction was short: pace as without one
    }
    const int64_t n = std::min<int64_t>(chunk, cap - queued);
    return (int)(n + (n & 1));
  }
  void queued_chunk(int n) {
    ++launched;
    queued += n;
  }
};

// pred: the previous solve's launch count, or 0 for none; chunk: launches
// per chunk (rounded down to even, at least 2). A solve never needs more than
// (max_refine + 1) inner solves of at most max_inner + 2 launches each.
inline Pacer make_pacer(int64_t max_inner, int64_t max_refine, int64_t pred,
                        int chunk = kChunk) {
  Pacer p;
  p.chunk = std::max(2, chunk & ~1);
  const int64_t max_launch = (max_refine + 1) * (max_inner + 2) + 2 * p.chunk;
  p.limit = (max_launch / p.chunk + 2) * p.chunk;
  p.cap = pred > 0 ? pred + kPredMargin : p.limit;
  return p;
}

}  // namespace fi
