// binary64 instantiation of the fused Sod stage kernel, and the dispatch.
#include "sod_stage.h"

namespace rsl {

int launch_stage_f64(int stage, int cls, const InstDesc* d, const StageClass* cl, char* fb, char* wb, hipStream_t s) {
    return launch_stage_any<double>(stage, cls, d, cl, fb, wb, s);
}

// Velocity-set classes of the stage kernel (see launch_cls).
int stage_class_of(int V) {
    if (V <= 4 * 8) return 0;
    if (V <= 4 * 16) return 1;
    if (V <= 8 * 16) return 2;
    if (V <= 8 * 2 * 16) return 3;
    if (V <= 8 * 2 * 20) return 4;
    return V <= 8 * 2 * 24 ? 5 : -1;
}

int stage_tile_cells(int cls) { return cls >= 3 ? 31 : 63; }

int launch_sod_stage(const InstDesc& d, int stage, hipStream_t s) {
    const int cls = stage_class_of(d.V);
    if (cls < 0) return set_error(RSL_EUNSUPPORTED, "Sod stage: more than 384 velocities");
    if (d.dtype == RSL_F64) return launch_stage_f64(stage, cls, &d, nullptr, nullptr, nullptr, s);
    return launch_stage_f32(stage, cls, &d, nullptr, nullptr, nullptr, s);
}

int launch_sod_class_stage(const StageClass& cl, int dtype, int stage, char* fbase, char* wbase, hipStream_t s) {
    if (cl.nitems == 0) return RSL_OK;
    if (dtype == RSL_F64) return launch_stage_f64(stage, cl.cls, nullptr, &cl, fbase, wbase, s);
    return launch_stage_f32(stage, cl.cls, nullptr, &cl, fbase, wbase, s);
}

}  // namespace rsl
