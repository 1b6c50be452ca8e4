// Instantiations of the elementwise kernel for 8-mode tensors (one
// translation unit per mode count, so they compile in parallel).
#include "ec_kernel.hpp"

namespace spt {

EcFnPtr pick_ec_n8(int rank, int fdtype, int words, int kind, bool reuse) {
    return pick_layout<8>(rank, fdtype, words, kind, reuse);
}

}  // namespace spt
