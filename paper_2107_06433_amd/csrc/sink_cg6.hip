// Instantiations of the fused Sinkhorn kernel with 64 column lane(s) per item.
#include "sink_kernel.h"

namespace wmd {

const SinkEntry* sink_table_cg6(int* n) {
  static const SinkEntry t[] = {WMD_SINK_TC(WMD_SINK_ENTRY, 2, 6) WMD_SINK_TC(WMD_SINK_ENTRY, 3, 6) WMD_SINK_TC(WMD_SINK_ENTRY, 4, 6) WMD_SINK_TC(WMD_SINK_ENTRY, 5, 6) WMD_SINK_TC(WMD_SINK_ENTRY, 6, 6) WMD_SINK_TC(WMD_SINK_ENTRY, 7, 6) WMD_SINK_TC(WMD_SINK_ENTRY, 8, 6) WMD_SINK_TC(WMD_SINK_ENTRY, 10, 6) WMD_SINK_TC(WMD_SINK_ENTRY, 12, 6) WMD_SINK_TC(WMD_SINK_ENTRY, 16, 6)};
  *n = (int)(sizeof(t) / sizeof(t[0]));
  return t;
}

}  // namespace wmd
