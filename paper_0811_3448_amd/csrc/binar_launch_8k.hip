// Launch sequences of the fixed-width and in-place sorts for 8-byte keys,
// keys only (every digit width, tile and offset scheme that is built).
#include "binar_host.h"

namespace binar {

template int launch_sort<8, false>(const Resolved &, const Work &, const Layout &, const uint32_t *, uint32_t,
                                uint32_t, hipStream_t);
template int launch_inplace<8, false>(const Resolved &, const Work &, const Layout &, char *, uint32_t,
                                   hipStream_t);

}  // namespace binar
