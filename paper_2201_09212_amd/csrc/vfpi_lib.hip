// Single translation unit of the V-FPI library: the parts share the setup
// kernels, so they are compiled together.
#include "api.hip"
#include "forward.hip"
#include "batched.hip"
#include "adjoint.hip"
#include "vnode.hip"
#include "noalloc.hip"
