// Runs build_ss_plan (csrc/ss_plan.h) on a matrix read from a file and writes
// the plan back, for the Python checks in test_ss_plan.py.
//   in:  int64 n, n_pad; int32 W, S, BS, threads; int32 xy[2n]; int32 ell[W * n_pad]
//   out: int32 ok, grid, max_region; int32 perm[n]; int32 blocks[grid * 8];
//        int64 nregion; int32 region[nregion]; int64 nlmat; uint16 lmat[nlmat]
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ss_plan.h"

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t n = 0, n_pad = 0;
  int32_t W = 0, S = 0, BS = 0, threads = 0;
  bool ok = std::fread(&n, 8, 1, f) == 1 && std::fread(&n_pad, 8, 1, f) == 1 &&
            std::fread(&W, 4, 1, f) == 1 && std::fread(&S, 4, 1, f) == 1 &&
            std::fread(&BS, 4, 1, f) == 1 && std::fread(&threads, 4, 1, f) == 1;
  if (!ok || n < 0 || n_pad < n) return 2;
  std::vector<int32_t> xy(2 * n), ell((size_t)W * n_pad);
  ok = std::fread(xy.data(), 4, xy.size(), f) == xy.size() &&
       std::fread(ell.data(), 4, ell.size(), f) == ell.size();
  std::fclose(f);
  if (!ok) return 2;
  fi::SsPlan plan;
  const int32_t built = fi::build_ss_plan(S, BS, n, xy.data(), ell.data(), n_pad, W, threads,
                                             fi::kPlanLocalMax - 1, plan);
  FILE* o = std::fopen(argv[2], "wb");
  if (!o) return 2;
  std::fwrite(&built, 4, 1, o);
  std::fwrite(&plan.grid, 4, 1, o);
  std::fwrite(&plan.max_region, 4, 1, o);
  if (built) {
    std::fwrite(plan.perm.data(), 4, plan.perm.size(), o);
    std::fwrite(plan.blocks.data(), sizeof(fi::BlockPlan), plan.blocks.size(), o);
    const int64_t nh = (int64_t)plan.region.size(), nl = (int64_t)plan.lmat.size();
    std::fwrite(&nh, 8, 1, o);
    std::fwrite(plan.region.data(), 4, plan.region.size(), o);
    std::fwrite(&nl, 8, 1, o);
    std::fwrite(plan.lmat.data(), 2, plan.lmat.size(), o);
  }
  std::fclose(o);
  return 0;
}
