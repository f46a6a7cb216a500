// binary32-storage instantiation of the fused Sod stage kernel.
#include "sod_split.h"

namespace rsl {

int launch_stage_f32(int stage, int var, const InstDesc* d, const StageClass* cl, char* fb, char* wb, hipStream_t s,
                     int seq) {
    return launch_stage_any<float>(stage, var, d, cl, fb, wb, s, seq);
}

}  // namespace rsl
