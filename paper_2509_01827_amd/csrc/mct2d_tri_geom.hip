// Crack-path geometry query of an unstructured mesh (Sec. 2.2, Figs. 2-2
// and 2-3): for every tip edge a of an element and every exit edge k the
// unit normal of the segment between the two edge midpoints, oriented
// toward node n_{a+1}, and its length, with the expressions the step uses
// (correctly rounded division and square root, no contraction).
#include <cmath>

#include "mct2d_tri.h"
#include "mct2d_tri_host.h"

namespace mct {
namespace tri {
namespace {

__device__ __forceinline__ int corner_node(const int4 &c, int n) {
    return n == 0 ? c.x : (n == 1 ? c.y : (n == 2 ? c.z : c.w));
}

// One thread per requested element: 36 values, [a][j][nx, ny, length] for
// a = 0..3 and exit edge k = a+1+j mod nv, j = 0..2; NaN where a or j does
// not exist (triangles: a = 3, j = 2).
__global__ void k_path_geometry(Params p, int n, const int32_t *elem, double *out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int4 c = p.conn[elem[t]];
    const int nv = p.nv;
    double *o = out + (int64_t)t * 36;
    for (int a = 0; a < 4; ++a)
        for (int j = 0; j < 3; ++j) {
            double *r = o + a * 9 + 3 * j;
            if (a >= nv || j >= nv - 1) {
                r[0] = r[1] = r[2] = NAN;
                continue;
            }
            const int k = (a + 1 + j) % nv;
            const double2 P0 = p.xy[corner_node(c, a)], P1 = p.xy[corner_node(c, (a + 1) % nv)];
            const double2 Q0 = p.xy[corner_node(c, k)], Q1 = p.xy[corner_node(c, (k + 1) % nv)];
            const double g0x = 0.5 * (P0.x + P1.x), g0y = 0.5 * (P0.y + P1.y);
            const double gkx = 0.5 * (Q0.x + Q1.x), gky = 0.5 * (Q0.y + Q1.y);
            const double dx = gkx - g0x, dy = gky - g0y;
            const double L = sqrt(dx * dx + dy * dy);
            double cx = dy / L, cy = -dx / L;
            if (cx * (P1.x - g0x) + cy * (P1.y - g0y) < 0.0) {
                cx = -cx;
                cy = -cy;
            }
            r[0] = cx;
            r[1] = cy;
            r[2] = L;
        }
}

}  // namespace

hipError_t launch_path_geometry(const Params &p, int n, const int32_t *elem, double *out, hipStream_t st) {
    (void)hipGetLastError();
    if (n > 0) k_path_geometry<<<(n + 255) / 256, 256, 0, st>>>(p, n, elem, out);
    return hipGetLastError();
}

}  // namespace tri
}  // namespace mct
