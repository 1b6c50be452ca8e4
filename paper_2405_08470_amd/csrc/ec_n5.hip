// Instantiations of the elementwise kernel for 5-mode tensors (one
// translation unit per mode count, so they compile in parallel).
#include "ec_kernel.hpp"

namespace spt {

EcFnPtr pick_ec_n5(int rank, int fdtype, int words, int kind, bool reuse) {
    return pick_layout<5>(rank, fdtype, words, kind, reuse);
}

}  // namespace spt
