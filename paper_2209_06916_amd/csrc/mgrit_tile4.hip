// Instances of the level-0 wavefront-tile kernel with 4 points per lane
// (float64, and float32 for the inner passes of mixed precision).
#include "mgrit_internal.h"

namespace mgrit {

namespace {

#include "mgrit_device.h"
#include "mgrit_tile.h"

}  // namespace

hipError_t launch_tiles_4(const LevelDesc *desc, const TileGeom &tg, const TileArgs &ta, hipStream_t stream) {
  return launch_tiles_p<4>(desc, tg, ta, stream);
}

hipError_t launch_tiles_4(const LevelDesc *desc, const TileGeom &tg, const TileArgs32 &ta, hipStream_t stream) {
  return launch_tiles_p<4>(desc, tg, ta, stream);
}

}  // namespace mgrit
