// Discrete divergence of a staggered velocity field: the right-hand side of
// the elliptic problem is built from div u* (paper, eq. ``elliptic``).
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
    A.f[e] = du * A.idx + dv / A.dyf[j] + dw * A.idz;
  }
}

hipError_t launch_divergence(const DivArgs& a, hipStream_t s) {
  const long n = (long)a.nx * a.ny * a.nz;
  long nb = (n + kThreads - 1) / kThreads;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_divergence, dim3((unsigned)nb), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace ibp
