// Batched stepping of many simulations (host side, private to the library):
// one descriptor per simulation and one block-to-simulation table per
// launch, laid out as one device image so that every step of every
// simulation in the batch is one launch per kernel class.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/lbm3.h"

namespace lbm3b {

struct Launch {
    int kind;                        // 0 moments, 1 ghost layers, 2 fused
    int D, prec, cls;                // kernel class
    size_t table_off;                // byte offset of its int table in the image
    std::vector<int> sims;           // simulations of this launch, in batch order
    std::vector<long long> prefix;   // prefix[k]: blocks of its first k simulations
};

struct Image {
    std::vector<unsigned char> bytes;  // device image: descriptors, then tables
    std::vector<Launch> launches;
    size_t desc_bytes = 0;
};

// Device bytes the image of these simulations takes (0 on invalid input).
size_t image_bytes(lbm3 *const *hs, int n);
// Descriptors and tables of hs[0..n-1] in this order, with the buffer
// parities the handles have now.
lbm3_status build(lbm3 *const *hs, int n, Image &img);
// Enqueue `steps` steps of hs[0..m-1] (a prefix of the order the image was
// built with) on `stream`, the image being at dev_base and `phase0` steps
// having been taken since it was built; advances the handles' state.
lbm3_status enqueue(lbm3 *const *hs, int m, const Image &img, const void *dev_base, int64_t phase0, int64_t steps,
                    hipStream_t stream);

}  // namespace lbm3b
