// cpf_internal.h -- host-side declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cpf_plan.h"

namespace cpf {

// Robot as the host keeps it: dof rows of DH parameters plus cos/sin of the
// twist computed once in double.
struct HostRobot {
    int dof;             // 7 or 8 joints
    double a[NJMAX], d[NJMAX], alpha[NJMAX], ca[NJMAX], sa[NJMAX], off[NJMAX], lo[NJMAX], hi[NJMAX];
    uint32_t prism;      // bit i set: joint i is prismatic
    bool has_caps;
    double cap[NJMAX][7];   // capsule of each link: p0, p1 (frame after the link), radius
};

// Plan geometry kinds, one LM and report kernel instance each: an
// all-revolute chain, collision capsules (always all-revolute), a chain with
// a prismatic joint.
enum { GEO_PLAIN = 0, GEO_COLL = 1, GEO_PRISM = 2, GEO_KINDS = 3 };
inline int plan_geo(const HostRobot &hr) { return hr.has_caps ? GEO_COLL : (hr.prism ? GEO_PRISM : GEO_PLAIN); }

// Capsules passed to a kernel by value (dof rows used).
struct HostCaps {
    double v[NJMAX][7];
};

// Chain lengths with kernels: 7 joints (namespace j7) and 8 (j8); dof_bit
// marks one in a set.
inline bool dof_supported(int dof) { return dof == 7 || dof == 8; }
inline int dof_bit(int dof) { return dof == 8 ? 2 : 1; }

namespace j7 {
#include "cpf_launch.inc"
}
namespace j8 {
#include "cpf_launch.inc"
}

// The launchers of the kernels built for `dof` joints.
#define CPF_BY_DOF(dof, call) ((dof) == 8 ? j8::call : j7::call)


}  // namespace cpf
