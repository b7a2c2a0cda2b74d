// Instantiations of the fused Sinkhorn kernel with 32 column lane(s) per item.
#include "sink_kernel.h"

namespace wmd {

const SinkEntry* sink_table_cg5(int* n) {
  static const SinkEntry t[] = {WMD_SINK_TC(WMD_SINK_ENTRY, 3, 5) WMD_SINK_TC(WMD_SINK_ENTRY, 4, 5) WMD_SINK_TC(WMD_SINK_ENTRY, 5, 5) WMD_SINK_TC(WMD_SINK_ENTRY, 6, 5) WMD_SINK_TC(WMD_SINK_ENTRY, 7, 5) WMD_SINK_TC(WMD_SINK_ENTRY, 8, 5)};
  *n = (int)(sizeof(t) / sizeof(t[0]));
  return t;
}

}  // namespace wmd
