// The general x and z transforms with every stage kind (radix-7 and
// radix-11 butterflies, direct-sum stages, Bluestein's convolution), and the
// entry points that pick a kernel family per plan: factorisations with
// radices 2, 3, 4, 5 and 8 only take the narrow family (ibp_xz_narrow.hip).
#include "ibp_xz_kernels.hpp"

namespace ibp {

IBP_XZ_FAMILY(extern, false)
IBP_XZ_FAMILY(, true)

template <typename T>
hipError_t launch_batch_xr2c(int mode, bool small, bool wide, const BatchGrid<T>* d, const long* start, long nblocks,
                             const BatchPtrs& p, const BatchLaunch& l, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  return wide ? batch_xr2c_w<T, true>(mode, small, d, start, nblocks, p, l, s)
              : batch_xr2c_w<T, false>(mode, small, d, start, nblocks, p, l, s);
}

template <typename T>
hipError_t launch_batch_xc2r(int mode, bool small, bool wide, const BatchGrid<T>* d, const long* start, long nblocks,
                             const BatchPtrs& p, const BatchLaunch& l, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  return wide ? batch_xc2r_w<T, true>(mode, small, d, start, nblocks, p, l, s)
              : batch_xc2r_w<T, false>(mode, small, d, start, nblocks, p, l, s);
}

template <typename T>
hipError_t launch_batch_zfft(bool inverse, bool small, bool wide, const BatchGrid<T>* d, const long* start,
                             long nblocks, const BatchLaunch& l, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  return wide ? batch_zfft_w<T, true>(inverse, small, d, start, nblocks, l, s)
              : batch_zfft_w<T, false>(inverse, small, d, start, nblocks, l, s);
}

template <typename T>
hipError_t launch_xr2c(int mode, bool small, bool wide, const XArgs<T>& a, hipStream_t s) {
  return wide ? xr2c_w<T, true>(mode, small, a, s) : xr2c_w<T, false>(mode, small, a, s);
}

template <typename T>
hipError_t launch_xc2r(int mode, bool small, bool wide, const XArgs<T>& a, hipStream_t s) {
  return wide ? xc2r_w<T, true>(mode, small, a, s) : xc2r_w<T, false>(mode, small, a, s);
}

template <typename T>
hipError_t launch_zfft(bool inverse, bool small, bool wide, const ZfArgs<T>& a, int nplanes, hipStream_t s) {
  return wide ? zfft_w<T, true>(inverse, small, a, nplanes, s) : zfft_w<T, false>(inverse, small, a, nplanes, s);
}

template hipError_t launch_batch_xr2c<double>(int, bool, bool, const BatchGrid<double>*, const long*, long,
                                              const BatchPtrs&, const BatchLaunch&, hipStream_t);
template hipError_t launch_batch_xr2c<float>(int, bool, bool, const BatchGrid<float>*, const long*, long,
                                             const BatchPtrs&, const BatchLaunch&, hipStream_t);
template hipError_t launch_batch_xc2r<double>(int, bool, bool, const BatchGrid<double>*, const long*, long,
                                              const BatchPtrs&, const BatchLaunch&, hipStream_t);
template hipError_t launch_batch_xc2r<float>(int, bool, bool, const BatchGrid<float>*, const long*, long,
                                             const BatchPtrs&, const BatchLaunch&, hipStream_t);
template hipError_t launch_batch_zfft<double>(bool, bool, bool, const BatchGrid<double>*, const long*, long,
                                              const BatchLaunch&, hipStream_t);
template hipError_t launch_batch_zfft<float>(bool, bool, bool, const BatchGrid<float>*, const long*, long,
                                             const BatchLaunch&, hipStream_t);
template hipError_t launch_xr2c<double>(int, bool, bool, const XArgs<double>&, hipStream_t);
template hipError_t launch_xr2c<float>(int, bool, bool, const XArgs<float>&, hipStream_t);
template hipError_t launch_xc2r<double>(int, bool, bool, const XArgs<double>&, hipStream_t);
template hipError_t launch_xc2r<float>(int, bool, bool, const XArgs<float>&, hipStream_t);
template hipError_t launch_zfft<double>(bool, bool, bool, const ZfArgs<double>&, int, hipStream_t);
template hipError_t launch_zfft<float>(bool, bool, bool, const ZfArgs<float>&, int, hipStream_t);

}  // namespace ibp
