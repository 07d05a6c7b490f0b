// The cube-to-ball map of mapped meshes, for host and device code.
//
// A mapped mesh is the BC octree of the reference cube [0,1]^3 pushed through a map Phi; the mesh's
// cells are the images of the reference cubes. The map here is the analytic cube-to-sphere mapping
// (reviewed by Zucker and Higashi, "Cube-to-sphere projections for procedural texturing and beyond",
// JCGT 7(2), 2018) applied to the whole volume: with u = 2 xi - 1,
//     y_i = u_i sqrt(1 - u_j^2 / 2 - u_k^2 / 2 + u_j^2 u_k^2 / 3),   Phi(xi) = (1 + y) / 2,
// which takes [0,1]^3 onto the ball of centre (1/2, 1/2, 1/2) and radius 1/2 (the cube's faces onto
// the sphere). D Phi(xi) = D y(u); its determinant is positive inside the cube and tends to zero at
// the cube's edges, where two faces meet on the smooth sphere.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace bcv {

// Phi(x) (3 values) and J(x) = det D Phi(x) for a reference point x in [0,1]^3.
__host__ __device__ inline void ball_map(const double x[3], double p[3], double *jac)
{
    double u[3], s[3], d[3][3];
    for (int i = 0; i < 3; ++i) u[i] = 2.0 * x[i] - 1.0;
    for (int i = 0; i < 3; ++i) {
        const int j = i == 2 ? 0 : i + 1, k = i == 0 ? 2 : i - 1;
        const double uj2 = u[j] * u[j], uk2 = u[k] * u[k];
        s[i] = sqrt(1.0 - 0.5 * (uj2 + uk2) + uj2 * uk2 * (1.0 / 3.0));
        p[i] = 0.5 + 0.5 * u[i] * s[i];
        const double h = u[i] / (2.0 * s[i]);
        d[i][i] = s[i];
        d[i][j] = h * u[j] * (2.0 * uk2 * (1.0 / 3.0) - 1.0);  // d y_i / d u_j
        d[i][k] = h * u[k] * (2.0 * uj2 * (1.0 / 3.0) - 1.0);
    }
    *jac = d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) - d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
           d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]);
}

}  // namespace bcv
