// Host check of the flux work decomposition: for a set of grid shapes and
// boundary conditions, every face of every direction must be taken by
// exactly one live lane slot of exactly one flux block (flux_block_counts,
// flux_block, face_of_block, banded_cell), and the index splitting must
// agree with integer division.  Prints "ok" or the first failure.
#include <cstdio>
#include <vector>

#include "box_kernels.h"

using namespace hgks;

static BoxGrid grid(int nx, int ny, int nz, int per) {
  BoxGrid G{};
  const int n[3] = {nx, ny, nz};
  for (int d = 0; d < 3; ++d) {
    G.n[d] = n[d];
    G.per[d] = (per >> d) & 1;
    G.g[d] = G.per[d] ? 0 : 1;
    G.nr[d] = n[d] + 2 * G.g[d];
  }
  for (int d = 0; d < 3; ++d) {
    for (int e = 0; e < 3; ++e) G.nf[d][e] = n[e];
    if (!G.per[d]) G.nf[d][d] += 1;
  }
  set_index_split(G);
  return G;
}

static bool check(const BoxGrid& G) {
  unsigned nb[3];
  flux_block_counts(G, nb);
  std::vector<int> seen[3];
  for (int d = 0; d < 3; ++d) seen[d].assign((size_t)G.nf[d][0] * G.nf[d][1] * G.nf[d][2], 0);
  const unsigned total = nb[0] + nb[1] + nb[2];
  std::vector<int> used[3];
  for (int d = 0; d < 3; ++d) used[d].assign(nb[d], 0);
  for (unsigned b = 0; b < total; ++b) {
    int D;
    unsigned lb;
    flux_block(b, nb, D, lb);
    if (D < 0 || D > 2 || lb >= nb[D] || used[D][lb]++) {
      printf("block %u -> (%d, %u) invalid or repeated\n", b, D, lb);
      return false;
    }
    for (unsigned slot = 0; slot < 64; ++slot) {
      int c[3];
      size_t f;
      const bool live = face_of_block(G, D, lb, slot, c, f);
      for (int e = 0; e < 3; ++e) {
        const int hi = G.n[e] + (e == D && !G.per[e] ? 1 : 0);
        if (c[e] < 0 || c[e] >= hi) {
          printf("face cell out of range: D %d lb %u slot %u axis %d value %d\n", D, lb, slot, e, c[e]);
          return false;
        }
      }
      const size_t expect = (size_t)c[0] + (size_t)G.nf[D][0] * ((size_t)c[1] + (size_t)G.nf[D][1] * c[2]);
      if (f != expect || f >= seen[D].size()) {
        printf("face index mismatch\n");
        return false;
      }
      if (live && seen[D][f]++) {
        printf("face %zu of direction %d taken twice\n", f, D);
        return false;
      }
    }
  }
  for (int d = 0; d < 3; ++d)
    for (size_t f = 0; f < seen[d].size(); ++f)
      if (seen[d][f] != 1) {
        printf("face %zu of direction %d not taken\n", f, d);
        return false;
      }
  // index splitting against integer division
  const uint32_t N = (uint32_t)G.nr[0] * G.nr[1] * G.nr[2];
  for (uint32_t k = 0; k < N; k += 1 + N / 5000) {
    int c0, c1, c2;
    split_index(k, G.nr[0], G.nr[1], G.inv_nr[0], G.inv_nr[1], c0, c1, c2);
    if (c0 != (int)(k % G.nr[0]) || c1 != (int)((k / G.nr[0]) % G.nr[1]) ||
        c2 != (int)(k / ((uint32_t)G.nr[0] * G.nr[1]))) {
      printf("split_index wrong at %u\n", k);
      return false;
    }
  }
  return true;
}

int main() {
  const int shapes[][3] = {{16, 16, 16}, {10, 9, 8}, {13, 7, 11}, {64, 3, 5}, {2, 2, 2}, {100, 37, 19},
                           {32, 48, 96}, {128, 17, 3}, {5, 40, 6}};
  for (const auto& s : shapes)
    for (int per = 0; per < 8; ++per)
      if (!check(grid(s[0], s[1], s[2], per))) {
        printf("failed for %d x %d x %d, periodic mask %d\n", s[0], s[1], s[2], per);
        return 1;
      }
  // split_index near the 32-bit limit
  const int e0 = 1625, e1 = 1621;
  const double i0 = div_inv(e0), i1 = div_inv(e1);
  for (uint64_t k = 4294967295ull; k > 4294967295ull - 200000; --k) {
    int c0, c1, c2;
    split_index((uint32_t)k, e0, e1, i0, i1, c0, c1, c2);
    if ((uint64_t)c0 != k % e0 || (uint64_t)c1 != (k / e0) % e1 || (uint64_t)c2 != k / ((uint64_t)e0 * e1)) {
      printf("split_index wrong near 2^32 at %llu\n", (unsigned long long)k);
      return 1;
    }
  }
  printf("ok\n");
  return 0;
}
