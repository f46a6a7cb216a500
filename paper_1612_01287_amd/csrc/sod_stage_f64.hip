// binary64 instantiation of the fused Sod stage kernel, and the dispatch.
#include "sod_split.h"

namespace rsl {

int launch_stage_f64(int stage, int var, const InstDesc* d, const StageClass* cl, char* fb, char* wb, hipStream_t s,
                     int seq) {
    return launch_stage_any<double>(stage, var, d, cl, fb, wb, s, seq);
}

bool stage_variant_shape(int var, int* W, int* NV, int* TW, int* form, int* WC) {
    switch (var) {
#define RSL_SHAPE(id, w, nv, tw) \
    case id: *W = w; *NV = nv; *TW = tw; *form = kFormFused; *WC = 0; return true;
        RSL_STAGE_VARIANTS(RSL_SHAPE)
#undef RSL_SHAPE
#define RSL_SHAPE(id, w, nv, wc) \
    case id: *W = w; *NV = nv; *TW = kLanes; *form = kFormSplit; *WC = wc; return true;
        RSL_SPLIT_VARIANTS(RSL_SHAPE)
#undef RSL_SHAPE
#define RSL_SHAPE(id, w, nv, wc, k) \
    case id: *W = w; *NV = nv; *TW = kLanes; *form = kFormLoop; *WC = wc; return true;
        RSL_LOOP_VARIANTS(RSL_SHAPE)
#undef RSL_SHAPE
        default: return false;
    }
}

int stage_variant_capacity(int var) {
    int W, NV, TW, WC, form;
    if (!stage_variant_shape(var, &W, &NV, &TW, &form, &WC)) return 0;
    return form != kFormFused ? kMaxVelocities : W * (kLanes / TW) * NV;
}

int stage_variant_tile_cells(int var) {
    int W, NV, TW, WC, form;
    return stage_variant_shape(var, &W, &NV, &TW, &form, &WC) ? TW - 1 : 0;
}

int stage_variant_count() {
    int n = 0, W, NV, TW, WC, form;
    while (stage_variant_shape(n, &W, &NV, &TW, &form, &WC)) ++n;
    return n;
}

// Default variant for a velocity set, and the batch class it belongs to.
static const int kDefaultVariant[kClasses] = {13, 13, 14, 14, 14, 14, 14};

// Largest V of each class (the last class takes every larger set).
static const int kClassMaxV[kClasses] = {32, 64, 128, 256, 320, 384, kMaxVelocities};

int stage_class_of(int V) {
    for (int c = 0; c < kClasses; ++c)
        if (V <= kClassMaxV[c]) return c;
    return -1;
}

int stage_default_variant(int cls) { return kDefaultVariant[cls]; }

int launch_sod_stage(const InstDesc& d, int stage, hipStream_t s, int seq) {
    const int cls = stage_class_of(d.V);
    if (cls < 0) return set_error(RSL_EUNSUPPORTED, "Sod stage: velocity set too large");
    const int var = kDefaultVariant[cls];
    if (d.dtype == RSL_F64) return launch_stage_f64(stage, var, &d, nullptr, nullptr, nullptr, s, seq);
    return launch_stage_f32(stage, var, &d, nullptr, nullptr, nullptr, s, seq);
}

int launch_sod_class_stage(const StageClass& cl, int dtype, int stage, char* fbase, char* wbase, hipStream_t s,
                           int seq) {
    if (cl.nitems == 0) return RSL_OK;
    if (dtype == RSL_F64) return launch_stage_f64(stage, cl.var, nullptr, &cl, fbase, wbase, s, seq);
    return launch_stage_f32(stage, cl.var, nullptr, &cl, fbase, wbase, s, seq);
}

}  // namespace rsl
