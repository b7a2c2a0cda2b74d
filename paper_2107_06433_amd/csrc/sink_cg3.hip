// Instantiations of the fused Sinkhorn kernel with 8 column lane(s) per item.
#include "sink_kernel.h"

namespace wmd {

const SinkEntry* sink_table_cg3(int* n) {
  static const SinkEntry t[] = {WMD_SINK_TC(WMD_SINK_ENTRY, 3, 3) WMD_SINK_TC(WMD_SINK_ENTRY, 4, 3) WMD_SINK_TC(WMD_SINK_ENTRY, 5, 3) WMD_SINK_TC(WMD_SINK_ENTRY, 6, 3) WMD_SINK_TC(WMD_SINK_ENTRY, 7, 3) WMD_SINK_TC(WMD_SINK_ENTRY, 8, 3)};
  *n = (int)(sizeof(t) / sizeof(t[0]));
  return t;
}

}  // namespace wmd
