// Implicit-explicit Sod steps (imex.hip): launchers and the work items of a
// batch.
#pragma once

#include <hip/hip_runtime.h>

#include "rsl_impl.h"

namespace rsl {

// Classes of velocity sets by the lanes each cell's implicit solve takes
// (Q_xi <= 4, 8, 16, 32, 64, 128, 256, 512, 1024).
constexpr int kImexClasses = 9;
int imex_class(int Q);
int imex_cells_per_item(int Q);   // cells of one batch implicit-stage workgroup
int imex_cells_per_explicit_item();   // cells of one batch explicit-pass workgroup

// Device item lists of a batch: per class (instance, first cell) of each
// implicit-stage workgroup, and (instance, first cell) of each explicit-pass
// workgroup.
struct ImexItems {
    const int2* items[kImexClasses];
    int n[kImexClasses];
    const int2* x;
    int nx;
};

// The CFL bound dt max|xi| / dz < 1 alone (the implicit-explicit steps' only
// step limit); RSL_EINVAL / RSL_EUNSTABLE with the message set.
int check_cfl(const rsl_quad* q, const rsl_problem* p, double dt);

int launch_imex_steps(const InstDesc& d, int dtype, int nsteps, hipStream_t s);
int launch_imex_batch_steps(const InstDesc* descs, const ImexItems& items, int dtype, char* fbase, char* wbase,
                            int nsteps, hipStream_t s);

}  // namespace rsl
