// Instantiations of the fused Sinkhorn kernel with 2 column lane(s) per item.
#include "sink_kernel.h"

namespace wmd {

const SinkEntry* sink_table_cg1(int* n) {
  static const SinkEntry t[] = {WMD_SINK_TC(WMD_SINK_ENTRY, 4, 1) WMD_SINK_TC(WMD_SINK_ENTRY, 6, 1) WMD_SINK_TC(WMD_SINK_ENTRY, 8, 1)};
  *n = (int)(sizeof(t) / sizeof(t[0]));
  return t;
}

}  // namespace wmd
