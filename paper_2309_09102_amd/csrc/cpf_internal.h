// cpf_internal.h -- host-side declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cpf_device.h"

namespace cpf {

// Robot as the host keeps it: DH rows plus cos/sin of the twist computed
// once in double.
struct HostRobot {
    double a[NJ], d[NJ], alpha[NJ], ca[NJ], sa[NJ], off[NJ], lo[NJ], hi[NJ];
    uint32_t prism;      // bit i set: joint i is prismatic
    bool has_caps;
    double cap[NJ][7];   // capsule of each link: p0, p1 (frame after the link), radius
};

// Plan geometry kinds, one LM and report kernel instance each: an
// all-revolute chain, collision capsules (always all-revolute), a chain with
// a prismatic joint.
enum { GEO_PLAIN = 0, GEO_COLL = 1, GEO_PRISM = 2, GEO_KINDS = 3 };
inline int plan_geo(const HostRobot &hr) { return hr.has_caps ? GEO_COLL : (hr.prism ? GEO_PRISM : GEO_PLAIN); }

// Capsules passed to a kernel by value.
struct HostCaps {
    double v[NJ][7];
};

// Kernel launchers (asynchronous on stream s).
hipError_t fk_batch_launch(const HostRobot &hr, int64_t M, int prec, const void *q, void *pose,
                           void *J, hipStream_t s);
// Collision distances (self, environment) of M configurations q [7][M] into
// dist [2][M], optionally gradients [14][M]; obs: device [n_obs][18].
hipError_t coll_batch_launch(const HostRobot &hr, const HostCaps &caps, int n_obs, const double *obs, int64_t M,
                             int prec, const void *q, void *dist, void *grad, hipStream_t s);
// Convert the caller arrays of one plan (candidates [K][T][7], doubles or
// floats, and targets [T][12] doubles, device-resident) into the device
// layout (cand float [T][7][K], targets [12][T]).  bad non-null: inputs the
// host has not checked; non-finite values are stored as 0 and set *bad.
hipError_t stage_launch(const void *cand_in, bool cand_f32, const double *tg_in, int T, int K, float *cand,
                        double *targets, int *bad, hipStream_t s);
// Appended candidates raw [K_add][T][7] doubles into columns k_off .. of the
// float [T][7][K] candidate array.
hipError_t stage_append_launch(const double *raw, int T, int K_add, int K, int k_off, float *cand,
                               hipStream_t s);
// mjac of every candidate plan (max over steps and joints of the change
// between consecutive waypoints), cand float [T][7][K] -> out double [K].
hipError_t cand_mjac_launch(const float *cand, int T, int K, double *out, hipStream_t s);
// Search for nplans plans in two launches: the node penalties (with coll,
// after the nodes' collision penalties) and predecessor lists over the whole
// GPU, then the stage recursion, back-tracking and seed gather, one
// workgroup per plan.
hipError_t dp_lists_launch(const DevPlan *d_plans, int nplans, int maxK, int maxT, bool coll, hipStream_t s);
hipError_t dp_stages_launch(const DevPlan *d_plans, int nplans, int maxK, hipStream_t s);
// Penalties and predecessor lists of one plan after candidates K_old..K-1
// were appended (the old nodes' penalties and lists already copied in).
hipError_t dp_append_launch(const DevPlan *d_plan, int K_old, int K, int T, bool coll, hipStream_t s);
// Up to `iters` LM iterations for each plan of precision prec (0 = mixed,
// 1 = FP64), objective kind sched and geometry kind geo (GEO_*); empty slots
// (T = 0) and plans of another precision or kind are skipped.  tick_budget
// > 0 (serving ticks) caps a plan of T waypoints at about
// tick_budget / (T + 330) iterations per launch (at least one).
hipError_t lm_launch(const DevPlan *d_plans, int nplans, int prec, int sched, int geo, int iters, hipStream_t s,
                     int tick_budget = 0);
// Pose error vs targets and mjac of the current trajectory (FP64 FK).  With
// only_finished, only plans that reached their iteration target (or failed)
// and have not been reported yet.
hipError_t eval_launch(const DevPlan *d_plans, int nplans, int only_finished, int geo, hipStream_t s);

// Trajectory [7][T] (device) into rows [T][7] (device).
hipError_t soa_rows_launch(const double *soa, int T, double *rows, hipStream_t s);

}  // namespace cpf
