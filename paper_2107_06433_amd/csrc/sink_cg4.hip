// Instantiations of the fused Sinkhorn kernel with 16 column lane(s) per item.
#include "sink_kernel.h"

namespace wmd {

const SinkEntry* sink_table_cg4(int* n) {
  static const SinkEntry t[] = {WMD_SINK_TC(WMD_SINK_ENTRY, 3, 4) WMD_SINK_TC(WMD_SINK_ENTRY, 4, 4) WMD_SINK_TC(WMD_SINK_ENTRY, 5, 4) WMD_SINK_TC(WMD_SINK_ENTRY, 6, 4) WMD_SINK_TC(WMD_SINK_ENTRY, 7, 4) WMD_SINK_TC(WMD_SINK_ENTRY, 8, 4)};
  *n = (int)(sizeof(t) / sizeof(t[0]));
  return t;
}

}  // namespace wmd
