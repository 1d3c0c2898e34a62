// Single translation unit of all device code, so that the batched launches
// (batch.hip) can call the per-block bodies of every stage kernel.
#include "bvh.hip"
#include "model.hip"
#include "render.hip"
#include "loss.hip"
#include "backward.hip"
#include "edges.hip"
#include "shadow_edges.hip"
#include "noalloc.hip"
#include "probe.hip"
