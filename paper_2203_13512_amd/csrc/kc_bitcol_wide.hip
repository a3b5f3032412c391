// kc_bitcol_wide.hip -- the BitCol listing kernels of the widest word classes
// (24 and 32 words with the bitmaps in LDS when counting, in device memory
// with per-vertex output; 48 and 64 words always in device memory), compiled
// apart from the narrower classes (kc_bitcol.hip) so that the two build in
// parallel.
#include "kc_bitcol.h"

int kc_resolve_list_wide(const ListArgs& a, int cls, int nw, bool pv, ListLaunch* L) {
  switch (cls) {
    case 6:
      return pv ? resolve_list_nw_dev<24, true>(a, nw, L) : resolve_list_nw<24, false>(a, nw, L);
    case 7:
      return pv ? resolve_list_nw_dev<32, true>(a, nw, L) : resolve_list_nw<32, false>(a, nw, L);
    case 8:
      return pv ? resolve_list_nw_dev<48, true>(a, nw, L) : resolve_list_nw_dev<48, false>(a, nw, L);
    case 9:
      return pv ? resolve_list_nw_dev<64, true>(a, nw, L) : resolve_list_nw_dev<64, false>(a, nw, L);
  }
  return KC_EUNSUPPORTED;
}
