// Kernels of the HGKS stage on a periodic hexahedral (vertex) grid, static
// or moving (Pan & Xu, Sec. 2 final part, Sec. 3 Eqs. (10)-(11), Remark 2).
#pragma once

#include "common.h"
#include "gks_flux.h"

namespace hgks {

// Per-cell geometry record (doubles): volume, centroid (3), second central
// moments xx, yy, zz, xy, yz, xz (6).
constexpr int kHexGeo = 10;

struct HexGrid {
  int n[3];
  double period[3];
};

inline void hex_setup(HexGrid& H, const int n[3], const double period[3]) {
  for (int d = 0; d < 3; ++d) {
    H.n[d] = n[d];
    H.period[d] = period[d];
  }
}

}  // namespace hgks
