// Instantiations of the fused Sinkhorn kernel with 4 column lane(s) per item.
#include "sink_kernel.h"

namespace wmd {

const SinkEntry* sink_table_cg2(int* n) {
  static const SinkEntry t[] = {WMD_SINK_TC(WMD_SINK_ENTRY, 3, 2) WMD_SINK_TC(WMD_SINK_ENTRY, 4, 2) WMD_SINK_TC(WMD_SINK_ENTRY, 5, 2) WMD_SINK_TC(WMD_SINK_ENTRY, 6, 2) WMD_SINK_TC(WMD_SINK_ENTRY, 7, 2) WMD_SINK_TC(WMD_SINK_ENTRY, 8, 2)};
  *n = (int)(sizeof(t) / sizeof(t[0]));
  return t;
}

}  // namespace wmd
