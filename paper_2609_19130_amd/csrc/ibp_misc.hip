// Discrete divergence of a staggered velocity field: the right-hand side of
// the elliptic problem is (div u* - q) / (alpha dt) (paper, eq. ``elliptic``).
// u[j][k][i] sits on the x face at x = i dx, w[j][k][i] on the z face at
// z = k dz (both periodic), v[j][k][i] on the y face yf[j] (ny+1 rows).
#include "ibp_internal.hpp"

namespace ibp {

__global__ __launch_bounds__(kThreads) void k_divergence(DivArgs A) {
  const long n = (long)A.nx * A.ny * A.nz;
  const long plane = (long)A.nx * A.nz;
  for (long e = (long)blockIdx.x * kThreads + threadIdx.x; e < n; e += (long)gridDim.x * kThreads) {
    const long j = e / plane;
    const long rem = e - j * plane;
    const int k = (int)(rem / A.nx);
    const int i = (int)(rem - (long)k * A.nx);
    const int ip = i + 1 == A.nx ? 0 : i + 1;
    const int kp = k + 1 == A.nz ? 0 : k + 1;
    const long rowb = e - i;
    const double du = A.u[rowb + ip] - A.u[e];
    const double dw = A.w[j * plane + (long)kp * A.nx + i] - A.w[e];
    const double dv = A.v[e + plane] - A.v[e];
    double d = du * A.idx + dv / A.dyf[j] + dw * A.idz;
    if (A.q) d -= A.q[e];
    A.f[e] = d * A.scale;
  }
}

// Projection of the provisional velocity and pressure update, one pass over
// the cells (paper, eqs. ``velsolen`` and ``pressure``):
//   u -= adt (phi[i] - phi[i-1]) / dx,   w -= adt (phi[k] - phi[k-1]) / dz,
//   v on face j (1 <= j < ny) -= adt (phi[j] - phi[j-1]) / dyc_j,
//   p += phi - visc L_h phi.
// Wall faces of v: unchanged at a Neumann wall; at a Dirichlet wall (phi = 0
// on the face) the one-sided gradient over the half cell.  Cell (j,k,i)
// updates the faces west, south and below it (plus the upper wall face when
// j = ny-1), so every face has one writer.
__global__ __launch_bounds__(kThreads) void k_project(ProjArgs A) {
  const long plane = (long)A.nx * A.nz;
  const long n = plane * A.ny;
  for (long e = (long)blockIdx.x * kThreads + threadIdx.x; e < n; e += (long)gridDim.x * kThreads) {
    const long j = e / plane;
    const long rem = e - j * plane;
    const int k = (int)(rem / A.nx);
    const int i = (int)(rem - (long)k * A.nx);
    const long rowb = e - i;
    const int im = i == 0 ? A.nx - 1 : i - 1, ip = i + 1 == A.nx ? 0 : i + 1;
    const int km = k == 0 ? A.nz - 1 : k - 1, kp = k + 1 == A.nz ? 0 : k + 1;
    const double c0 = A.phi[e];
    const double xm = A.phi[rowb + im], xp = A.phi[rowb + ip];
    const double zm = A.phi[j * plane + (long)km * A.nx + i], zp = A.phi[j * plane + (long)kp * A.nx + i];
    const double ym = j > 0 ? A.phi[e - plane] : 0.0;          // wall value 0 beyond a wall
    const double yp = j + 1 < A.ny ? A.phi[e + plane] : 0.0;
    A.u[e] -= A.adt * (c0 - xm) * A.idx;
    A.w[e] -= A.adt * (c0 - zm) * A.idz;
    if (j > 0)
      A.v[e] -= A.adt * (c0 - ym) / A.dyc[j];
    else if (A.dir_lo)
      A.v[e] -= A.adt * (c0 - 0.0) / (0.5 * A.dyf[0]);
    if (j + 1 == A.ny && A.dir_hi) A.v[e + plane] -= A.adt * (0.0 - c0) / (0.5 * A.dyf[j]);
    if (A.p) {
      const double lap = (xp - 2.0 * c0 + xm) * A.idx * A.idx + (zp - 2.0 * c0 + zm) * A.idz * A.idz +
                         A.ya[j] * (ym - c0) + A.yc[j] * (yp - c0);
      A.p[e] += c0 - A.visc * lap;
    }
  }
}

hipError_t launch_project(const ProjArgs& a, hipStream_t s) {
  const long n = (long)a.nx * a.ny * a.nz;
  long nb = (n + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_project, dim3((unsigned)nb), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_divergence(const DivArgs& a, hipStream_t s) {
  const long n = (long)a.nx * a.ny * a.nz;
  long nb = (n + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_divergence, dim3((unsigned)nb), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace ibp
