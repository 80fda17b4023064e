// Row blocks with halos for the s-step CG launch (plain C++, no device code).
//
// The s-step launch advances S iterations of Jacobi PCG per launch. Each
// block applies the preconditioned operator S times to its rows' vectors, so
// it needs the rows within S hops of its own in the matrix graph. The free
// rows are therefore renumbered along a Hilbert curve over their lattice
// coordinates (the last lattice row and column clamped onto the one before),
// so that a block's BS consecutive rows form a compact patch and consecutive
// blocks are neighbouring patches (a block's halo rows mostly belong to
// blocks just before or after it, which run at about the same time on the
// same XCD: its cache still holds them), and each block gets:
//   - its region: its own rows (local index 0 .. nown-1), then the rows at
//     graph distance 1, 2, ..., S from them (ascending within each ring),
//     listed in full (own rows included) so that a region row is one load;
//   - a local matrix for the rows of its region at distance <= S - 1: for
//     each such row, 6 entries, each the neighbour's slot (bits 0-13: its
//     local index + 1; slot 0 is a zero the launch keeps in front of its
//     region values, so every entry is one unconditional load), bit 15 for
//     weight -1 (clear: -1/2), bit 14 marking padding (slot 0, weight bit
//     clear). On the quadtree mesh every off-diagonal entry of K_FF is -1/2
//     or -1, and no row has more than 6 of them (every mask measured; a
//     mesh with a longer row keeps the one-iteration launch).
// Rows of a block are [b * BS, min(n, (b + 1) * BS)) in the new order.
//
// Inputs come from the library's column-major ELL of K_FF (natural order):
// slot k of row i at ell[k * n_pad + i], column in bits 0-29, bit 30 padding,
// bit 31 weight -1.
#pragma once

#include <algorithm>
#include <cstdint>
#include <memory>
#include <vector>

#include "host_pool.h"

namespace fi {

constexpr int kPlanLocalBits = 14;
constexpr int32_t kPlanLocalMax = 1 << kPlanLocalBits;  // slots: region rows per block + 1, at most
constexpr uint16_t kPlanPad = 1u << 14;
constexpr uint16_t kPlanMinusOne = 1u << 15;
constexpr int kPlanSlots = 6;  // entries per local matrix row (12 bytes)

struct BlockPlan {
  int32_t reg_off;   // first region row of the block in SsPlan::region (0 when empty)
  int32_t lmat_off;  // first local matrix row of the block in SsPlan::lmat (0 when empty)
  int32_t nown;      // own rows
  int32_t n1;        // region rows at distance <= 1
  int32_t ninner;    // region rows at distance <= S - 1 (rows of the local matrix)
  int32_t nreg;      // region rows in all (distance <= S)
  int32_t pad0, pad1;
};
static_assert(sizeof(BlockPlan) == 32, "block table layout");

struct SsPlan {
  int S = 0, BS = 0;
  int64_t n = 0;
  int32_t grid = 0;              // blocks (a multiple of 8)
  int32_t max_region = 0;        // largest nreg over the blocks
  HostVec<int32_t> perm;         // new index -> natural row
  std::vector<BlockPlan> blocks;
  HostVec<int32_t> region;       // region rows (new indices), block after block
  HostVec<uint16_t> lmat;        // local matrix rows, kPlanSlots entries each
};

// Position of (x, y) along the Hilbert curve over [0, 2^order)^2: the
// quadrant digits from the top level down, each level's frame rotated or
// reflected so that consecutive positions are edge neighbours.
inline uint64_t hilbert_key(uint32_t x, uint32_t y, int order) {
  const uint32_t side = 1u << order;
  uint64_t d = 0;
  for (uint32_t s = side >> 1; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
    d += (uint64_t)s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = side - 1 - x;
        y = side - 1 - y;
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}

// Builds the plan. xy: lattice coordinates of the free rows (natural order,
// 2 per row); ell: the ELL copy described above (W slots). Returns false if
// a region exceeds max_region rows (below kPlanLocalMax) or a row has more
// than kPlanSlots entries (the caller then keeps the one-iteration launch).
// Each pass is split into `threads` tasks that run on the host pool; the
// plan does not depend on that number.
inline bool build_ss_plan(int S, int BS, int64_t n, const int32_t* xy, const int32_t* ell,
                          int64_t n_pad, int W, int threads, int max_region, SsPlan& out) {
  out = SsPlan{};
  out.S = S;
  out.BS = BS;
  out.n = n;
  if (n <= 0 || W > kPlanSlots || S < 1 || max_region >= kPlanLocalMax || max_region < BS)
    return false;
  // Hilbert order of the free rows. The lattice runs from 0 to N (a power of
  // two), and its last row and column would take a level of their own in the
  // key, which would string them out into blocks that are thin strips with wide
  // halos; coordinates are therefore clamped to N - 1, which keeps those
  // vertices next to their neighbours (ties go to the lower natural row).
  int32_t maxc = 0;
  for (int64_t i = 0; i < 2 * n; ++i) maxc = std::max(maxc, xy[i]);
  uint32_t top = 1;
  while (maxc > 1 && top * 2 <= (uint32_t)maxc) top *= 2;
  const uint32_t clampc = maxc > 1 ? top - 1 : (uint32_t)maxc;
  int order = 0;
  while (order < 31 && (1u << order) <= clampc) ++order;
  const int nthr = std::max(1, threads);
  auto range = [&](int t, int nt) {
    return std::pair<int64_t, int64_t>(n * t / nt, n * (t + 1) / nt);
  };
  // (key, row) pairs, key in the high 32 bits (keys take 2 bits per
  // coordinate bit, coordinates stay below 2^14)
  HostVec<uint64_t> kr(n);
  std::vector<uint64_t> tmax(nthr, 0);
  pool_run(nthr, [&](int64_t t, int64_t nt) {
    const auto [i0, i1] = range(t, nt);
    uint64_t m = 0;
    for (int64_t i = i0; i < i1; ++i) {
      const uint64_t k = hilbert_key(std::min((uint32_t)xy[2 * i], clampc),
                                     std::min((uint32_t)xy[2 * i + 1], clampc), order);
      m = std::max(m, k);
      kr[i] = (k << 32) | (uint64_t)i;
    }
    tmax[t] = m;
  });
  const uint64_t kmax = *std::max_element(tmax.begin(), tmax.end());
  if (kmax >> 32) return false;
  // stable least-significant-digit radix sort of the pairs by key (11 bits
  // a pass), so equal keys keep the natural order: each of the nthr chunks
  // counts its digits, and scatters its pairs in order after the pairs of
  // lower digits and of earlier chunks with the same digit
  {
    HostVec<uint64_t> b(n);
    std::vector<int64_t> cnt((size_t)nthr << 11);
    for (int shift = 32; shift == 32 || (kmax >> (shift - 32)) != 0; shift += 11) {
      pool_run(nthr, [&](int64_t t, int64_t nt) {
        const auto [i0, i1] = range((int)t, (int)nt);
        int64_t* c = &cnt[(size_t)t << 11];
        std::fill(c, c + 2048, 0);
        for (int64_t i = i0; i < i1; ++i) ++c[(kr[i] >> shift) & 2047];
      });
      int64_t sum = 0;
      for (int d = 0; d < 2048; ++d)
        for (int t = 0; t < nthr; ++t) {
          int64_t& c = cnt[((size_t)t << 11) + d];
          const int64_t v = c;
          c = sum;
          sum += v;
        }
      pool_run(nthr, [&](int64_t t, int64_t nt) {
        const auto [i0, i1] = range((int)t, (int)nt);
        int64_t* c = &cnt[(size_t)t << 11];
        for (int64_t i = i0; i < i1; ++i) b[c[(kr[i] >> shift) & 2047]++] = kr[i];
      });
      kr.swap(b);
    }
  }
  out.perm.resize(n);
  HostVec<int32_t> inv(n);
  pool_run(nthr, [&](int64_t t, int64_t nt) {
    const auto [i0, i1] = range((int)t, (int)nt);
    for (int64_t i = i0; i < i1; ++i) {
      const int32_t r = (int32_t)(kr[i] & 0xFFFFFFFFu);
      out.perm[i] = r;
      inv[r] = (int32_t)i;
    }
  });
  // neighbours in the new order: column (new index) and weight code, by
  // natural rows (the ELL is read in order; each row's list lands at its
  // new index)
  std::unique_ptr<int32_t[]> nbp(new int32_t[(size_t)n * kPlanSlots]);
  std::unique_ptr<uint8_t[]> nbwp(new uint8_t[(size_t)n * kPlanSlots]);
  int32_t* const nb = nbp.get();
  uint8_t* const nbw = nbwp.get();
  pool_run(nthr, [&](int64_t t, int64_t nt) {
    const auto [r0, r1] = range((int)t, (int)nt);
    for (int64_t r = r0; r < r1; ++r) {
      const size_t o = (size_t)inv[r] * kPlanSlots;
      int c = 0;
      for (int k = 0; k < W; ++k) {
        const int32_t e = ell[(size_t)k * n_pad + r];
        if (e & 0x40000000) continue;
        nb[o + c] = inv[e & 0x3FFFFFFF];
        nbw[o + c] = e < 0 ? 1 : 0;
        ++c;
      }
      for (; c < kPlanSlots; ++c) {
        nb[o + c] = -1;
        nbw[o + c] = 0;
      }
    }
  });
  const int64_t nblk = (n + BS - 1) / BS;
  out.grid = (int32_t)((nblk + 7) / 8 * 8);
  out.blocks.assign(out.grid, BlockPlan{});
  // per block: region (BFS by rings) and local matrix, built in parallel
  struct Part {
    std::vector<int32_t> region;
    std::vector<uint16_t> lmat;
    bool ok = true;
  };
  std::vector<Part> parts(out.grid);
  auto work = [&](int64_t t, int64_t nt) {
    // region membership: open addressing over new indices (row -> local
    // index), twice the largest region, cleared after each block
    constexpr uint32_t kTab = 2u * (uint32_t)kPlanLocalMax;
    std::vector<int32_t> tkey(kTab, -1), tval(kTab, -1);
    std::vector<uint32_t> used;
    auto slot = [&](int32_t row) {
      uint32_t h = ((uint32_t)row * 2654435761u) & (kTab - 1);
      while (tkey[h] != -1 && tkey[h] != row) h = (h + 1) & (kTab - 1);
      return h;
    };
    std::vector<int32_t> next;
    for (int64_t b = t; b < nblk; b += nt) {
      Part& P = parts[b];
      BlockPlan& B = out.blocks[b];
      const int64_t r0 = b * BS, r1 = std::min<int64_t>(n, r0 + BS);
      std::vector<int32_t> reg;
      auto add = [&](int32_t row) {
        const uint32_t h = slot(row);
        if (tkey[h] == row) return;
        tkey[h] = row;
        tval[h] = (int32_t)reg.size();
        used.push_back(h);
        reg.push_back(row);
      };
      for (int64_t i = r0; i < r1; ++i) add((int32_t)i);
      B.nown = (int32_t)(r1 - r0);
      size_t ring_lo = 0;
      for (int d = 1; d <= S && P.ok; ++d) {
        next.clear();
        const size_t ring_hi = reg.size();
        for (size_t q = ring_lo; q < ring_hi; ++q) {
          const int64_t i = reg[q];
          for (int k = 0; k < kPlanSlots; ++k) {
            const int32_t c = nb[(size_t)i * kPlanSlots + k];
            if (c >= 0 && tkey[slot(c)] != c) {
              const uint32_t h = slot(c);
              tkey[h] = c;  // reserve; the local index is set below, in ring order
              used.push_back(h);
              next.push_back(c);
              if (reg.size() + next.size() > (size_t)max_region) {
                P.ok = false;
                break;
              }
            }
          }
          if (!P.ok) break;
        }
        std::sort(next.begin(), next.end());
        ring_lo = reg.size();
        for (int32_t c : next) {
          tval[slot(c)] = (int32_t)reg.size();
          reg.push_back(c);
        }
        if (d == 1) B.n1 = (int32_t)reg.size();
        if (d == S - 1) B.ninner = (int32_t)reg.size();
      }
      if (S == 1) B.ninner = B.nown;
      B.nreg = (int32_t)reg.size();
      if (P.ok) {
        P.region.assign(reg.begin(), reg.end());
        P.lmat.assign((size_t)B.ninner * kPlanSlots, 0);
        for (int32_t l = 0; l < B.ninner; ++l) {
          const int64_t i = reg[l];
          for (int k = 0; k < kPlanSlots; ++k) {
            const int32_t c = nb[(size_t)i * kPlanSlots + k];
            uint16_t e = kPlanPad;  // the zero slot
            if (c >= 0)
              e = (uint16_t)((uint16_t)(tval[slot(c)] + 1) |
                             (nbw[(size_t)i * kPlanSlots + k] ? kPlanMinusOne : 0));
            P.lmat[(size_t)l * kPlanSlots + k] = e;
          }
        }
      }
      for (uint32_t h : used) {
        tkey[h] = -1;
        tval[h] = -1;
      }
      used.clear();
    }
  };
  pool_run(std::min<int64_t>(nthr, nblk), work);
  int64_t roff = 0, loff = 0;
  for (int32_t b = 0; b < out.grid; ++b) {
    if (!parts[b].ok) return false;
    BlockPlan& B = out.blocks[b];
    // an empty block points at the start of both lists (valid, unused rows)
    B.reg_off = B.nreg > 0 ? (int32_t)roff : 0;
    B.lmat_off = B.ninner > 0 ? (int32_t)loff : 0;
    roff += (int64_t)parts[b].region.size();
    loff += B.ninner;
    out.max_region = std::max(out.max_region, B.nreg);
    if (roff > INT32_MAX || loff > INT32_MAX / kPlanSlots) return false;
  }
  // the device memory a plan may take is bounded (region and local matrix
  // rows at most three per free row), so memory can be reserved before it
  // is built
  if (roff > 3 * n || loff > 3 * n) return false;
  out.region.resize(roff);
  out.lmat.resize((size_t)loff * kPlanSlots);
  pool_run(std::min<int64_t>(nthr, nblk), [&](int64_t t, int64_t nt) {
    for (int64_t b = t; b < nblk; b += nt) {
      const BlockPlan& B = out.blocks[b];
      std::copy(parts[b].region.begin(), parts[b].region.end(), out.region.begin() + B.reg_off);
      std::copy(parts[b].lmat.begin(), parts[b].lmat.end(),
                out.lmat.begin() + (size_t)B.lmat_off * kPlanSlots);
    }
  });
  return true;
}

}  // namespace fi
