// fields_f64.hip -- the FP64 instantiations of the field kernels of
// fields.hip, compiled apart so that they get their own instruction
// scheduling.  The FP64 field step holds two waves per SIMD (about 250
// VGPRs) and waits on memory for much of its time; the compiler's max-ilp scheduling
// strategy (build.py passes -amdgpu-sched-strategy=max-ilp for this file
// only) interleaves its independent loads and arithmetic further and takes
// about 3 % off the step.  The same strategy makes the FP32 field step and
// the pushes slower, so they keep the default.
#define GL_FIELDS_FP64
#include "fields.hip"
