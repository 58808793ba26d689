// Batched persistent launch (plans) and its tile-cost tuner.
#pragma once

#include "common.h"

namespace rise {

struct PlanImpl;
rise_status plan_build(PlanImpl** out, const rise_gemm_problem* g, int ng,
                       const rise_stencil_problem* st, int ns, const char* tune_path,
                       int forced_kind, hipStream_t stream);
rise_status plan_launch(PlanImpl* p, hipStream_t s);
rise_status plan_launch_direct(PlanImpl* p, hipStream_t s);
void rise_plan_free(PlanImpl* p);
int plan_items(const PlanImpl* p);
int plan_grid(const PlanImpl* p);
double plan_estimate(const PlanImpl* p);
int plan_kind(const PlanImpl* p, int i);
const char* kind_name(int k);
int num_kinds();
int kind_is_stencil(int k);
int kind_stencil_side(int k);
int kind_dtype(int k);
int kind_opb(int k);
// (bm, bn, bk) a GEMM tile kind runs; all zero for stencil kinds
rise_tile kind_tile(int k);

}  // namespace rise
