// Launch table of the compact register-resident panel kernel (gj_panel_rot_kernel):
// one instantiation per scalar type, panel width, rows per thread and thread count.
// Kept in a translation unit of its own so that it compiles beside the engine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/hss.h"
#include "common.hpp"
#include "k_gj.hpp"
#include "panel.hpp"

namespace hss {

// Arithmetic of the pivot search: single precision for double-precision matrices
// (gj_panel_rot_kernel explains why the pivot order needs no more).
template <class X> struct Search { using type = X; };
template <> struct Search<double> { using type = float; };
template <> struct Search<cd> { using type = cf; };

template <class X>
bool panel_rot_config(int rows, PanelShape& s) {
  // 16-column panels, up to four rows per thread
  if (rows <= 128) {
    s = {16, 1, 128};
    return true;
  }
  if (rows <= 256 * 4) {
    s = {16, (rows + 255) / 256, 256};
    return true;
  }
  if (rows <= 512 * 4) {
    s = {16, (rows + 511) / 512, 512};
    return true;
  }
  // real types search in single precision: up to eight rows per thread
  if (!traits<X>::cplx && rows <= 512 * 8) {
    const int rpt = (rows + 511) / 512;
    s = {16, rpt <= 6 ? 6 : 8, 512};
    return true;
  }
  return false;
}

template <class X>
void launch_panel_rot(const GjDesc<X>* dd, int nn, int j0, int nb, const PanelShape& s, hipStream_t st) {
  using S = typename Search<X>::type;
#define HSS_ROT(NB_, RPT_, NT_)                                                      \
  if (s.nb == NB_ && s.rpt == RPT_ && s.nt == NT_) {                                 \
    gj_panel_rot_kernel<X, NB_, RPT_, NT_, S><<<nn, NT_, 0, st>>>(dd, j0, nb);       \
    return;                                                                          \
  }
  HSS_ROT(16, 1, 128)
  HSS_ROT(16, 1, 256) HSS_ROT(16, 2, 256) HSS_ROT(16, 3, 256) HSS_ROT(16, 4, 256)
  HSS_ROT(16, 3, 512) HSS_ROT(16, 4, 512)
  if constexpr (!traits<X>::cplx) {
    HSS_ROT(16, 6, 512) HSS_ROT(16, 8, 512)
  }
#undef HSS_ROT
  throw Error(HSS_EDEVICE, "no panel variant for nb " + std::to_string(s.nb) + ", rpt " + std::to_string(s.rpt) +
                               ", threads " + std::to_string(s.nt));
}

template bool panel_rot_config<float>(int, PanelShape&);
template bool panel_rot_config<double>(int, PanelShape&);
template bool panel_rot_config<cf>(int, PanelShape&);
template bool panel_rot_config<cd>(int, PanelShape&);
template void launch_panel_rot<float>(const GjDesc<float>*, int, int, int, const PanelShape&, hipStream_t);
template void launch_panel_rot<double>(const GjDesc<double>*, int, int, int, const PanelShape&, hipStream_t);
template void launch_panel_rot<cf>(const GjDesc<cf>*, int, int, int, const PanelShape&, hipStream_t);
template void launch_panel_rot<cd>(const GjDesc<cd>*, int, int, int, const PanelShape&, hipStream_t);

}  // namespace hss
