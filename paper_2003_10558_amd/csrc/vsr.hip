// libvsr: the single translation unit of the HIP library (gfx950).
//   map.hpp     perspective vector map + tile caps      (step 1)
//   setup.hpp   per-triangle setup, ordering, cap index (step 2)
//   raster.hpp  conservative binning + rasterizer       (steps 3, 4)
//   submit.hpp  batched views                           (step 5)
//   api.hpp     C ABI (include/vsr.h)
#include "api.hpp"
