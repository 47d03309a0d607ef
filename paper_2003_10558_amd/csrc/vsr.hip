// libvsr: the single translation unit of the HIP library (gfx950).
//   map.hpp     perspective vector maps + tile caps     (step 1; sections 2.1-2.3)
//   setup.hpp   per-triangle setup, ordering, cap index (step 2)
//   gather.hpp  candidate gathering from the cap index  (step 3)
//   bin.hpp     conservative binning, two shapes        (step 3)
//   raster.hpp  rasterizer                              (step 4)
//   fused.hpp   depth-sliced bin + raster in one kernel (steps 3, 4)
//   submit.hpp  batched views                           (step 5)
//   resolve.hpp fragment data from barycentrics         (section 1.1.4)
//   aa.hpp      aliasing-free coverage, particles       (sections 1.1.1, 1.1.2, 1.3, 1.4)
//   wire.hpp    aliasing-free wire frame                (section 1.2)
//   api.hpp     C ABI (include/vsr.h)
//   noalloc.hpp vsr_render with a library-held scratch array
#include "api.hpp"
#include "noalloc.hpp"
