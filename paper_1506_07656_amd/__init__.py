"""MI355X DeepMatching: HIP kernels behind a C ABI (libdm.so) with a thin
Python binding.  See include/dm.h for the library contract."""
from .binding import (Batch, BatchInfo, BatchTiles, Pair, DMPyramid, DeepFlow, FlowInfo, FlowParams, GradPlan, InvariantInfo,
                      Pyramid, deepflow, flow_params, flow_plan, plan_grad,
                      top_loss, DM_BF16, DM_ENTRIES_LOCAL_MAXIMA, DM_ENTRIES_TOP, DM_FP32, DM_FP64, DMError,
                      DM_SCORE_PATH_SUM, DM_SCORE_START_END,
                      LIB_PATH, Match, Matcher, NOALLOC_MAX_BYTES, Params, PlanInfo, descriptors, lib,
                      match_descriptors, match_images, match_images_noalloc, match_invariant, params, plan,
                      plan_invariant, timing_enable, timing_read, version, workspace, workspace_views)

__all__ = ["Batch", "BatchInfo", "BatchTiles", "Pair", "DMPyramid", "DeepFlow", "FlowInfo", "FlowParams", "GradPlan",
           "InvariantInfo", "Pyramid", "deepflow", "flow_params", "flow_plan",
           "plan_grad", "top_loss", "DM_BF16", "DM_ENTRIES_LOCAL_MAXIMA", "DM_ENTRIES_TOP", "DM_FP32", "DM_FP64",
           "DM_SCORE_PATH_SUM", "DM_SCORE_START_END",
           "DMError", "LIB_PATH", "Match", "Matcher", "NOALLOC_MAX_BYTES", "Params", "PlanInfo", "descriptors",
           "lib", "match_descriptors", "match_images", "match_images_noalloc", "match_invariant", "params", "plan",
           "plan_invariant", "timing_enable", "timing_read", "version", "workspace", "workspace_views"]
