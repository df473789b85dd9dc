// GEMM autotuner (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "internal.h"

namespace tnrcs {

// Times the valid tile / split variants of GEMM step g (dtype TN_DTYPE_*)
// on its buffers (a, b, c; w: split workspace of g.split_max slabs or NULL;
// slot: magnitude record for scaled storage) on the null stream and sets
// g.tile and g.split_k to the fastest.  Synchronous.  db: optional cache file.
int tune_gemm(int dtype, GemmOp& g, const void* a, const void* b, void* c, float2* w, float* slot, const char* db,
              std::string& err);

// Kernel-class choices of whole steps, keyed by dtype and a canonical
// description of the step's operand layouts: lookup (process cache, then the
// database file db if given) and store (both).
bool class_lookup(int dtype, const std::string& key, const char* db, int* cls);
void class_store(int dtype, const std::string& key, const char* db, int cls, float ms);

}  // namespace tnrcs
