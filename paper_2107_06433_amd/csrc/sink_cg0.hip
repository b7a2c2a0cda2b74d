// Instantiations of the fused Sinkhorn kernel with 1 column lane(s) per item.
#include "sink_kernel.h"

namespace wmd {

const SinkEntry* sink_table_cg0(int* n) {
  static const SinkEntry t[] = {WMD_SINK_TC(WMD_SINK_ENTRY, 4, 0) WMD_SINK_TC(WMD_SINK_ENTRY, 8, 0)};
  *n = (int)(sizeof(t) / sizeof(t[0]));
  return t;
}

}  // namespace wmd
