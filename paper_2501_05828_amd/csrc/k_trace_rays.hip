// Explicit rays with an event log (ur_trace_rays): the k_trace_rays kernel of
// k_trace.hip, compiled in a translation unit of its own so that it can be
// built without loop unrolling.  Built with it (-O2 and above), a call with
// many rays dropped some direct-hit records in lanes whose direct-hit test
// held (a test of coplanar and coincident triangles found it); built without
// it, or at -O1, every record is there.  The kernels of the timed path are
// exact on the same scenes and keep their build.
#define UR_TRACE_RAYS_ONLY
#include "k_trace.hip"
