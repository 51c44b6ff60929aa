// Far field of the voxel polarisation (the radiated field of Sec. II's
// current distribution, as used for the RCS comparisons of Sec. III):
//   F(rhat) = (I - rhat rhat) sum_n P_n dV exp(+j k0 rhat . r_n),
// r_n the voxel centre relative to the grid centre; for the face unknowns of
// the rooftop discretisation (`faces`) component c of entry n sits half a
// cell further along axis c, which multiplies its phase factor by the
// direction's constant exp(+j k0 rhat_c d_c / 2).  Each workgroup sums a
// chunk of voxels for one direction (FP64 phases and sums); a second kernel
// adds the chunks of each direction in a fixed order (deterministic).
#include <stdexcept>
#include <string>

#include "krylov_dev.h"

namespace vie {

constexpr int FF_T = 256;          // threads per workgroup
constexpr int FF_CHUNK = 2048;     // voxels per workgroup

// Partial sums of the far field that allocates nothing (6 doubles per
// direction and voxel chunk): a fixed array of 8 MiB on every GPU the
// library runs on, held until the process ends.  Host code never uses the
// name itself (it is a host-side stand-in there): far_field_scratch_address
// returns the device's own address of its copy.
constexpr int64_t kFarScratchDoubles = int64_t(1) << 20;
static __device__ __align__(256) double scratch[kFarScratchDoubles];

__global__ void __launch_bounds__(FF_T) k_far_partial(const c128* P, int nx, int ny, int nz, double dx, double dy,
                                                      double dz, double k0, const double* rhat, int nchunk,
                                                      double* part, int faces) {
  const int dir = blockIdx.x / nchunk, chunk = blockIdx.x - dir * nchunk;
  const double rx = rhat[3 * dir], ry = rhat[3 * dir + 1], rz = rhat[3 * dir + 2];
  double hs[3] = {0.0, 0.0, 0.0}, hc[3] = {1.0, 1.0, 1.0};   // half-cell phase of each component
  if (faces) {
    sincos(0.5 * k0 * rx * dx, &hs[0], &hc[0]);
    sincos(0.5 * k0 * ry * dy, &hs[1], &hc[1]);
    sincos(0.5 * k0 * rz * dz, &hs[2], &hc[2]);
  }
  const int64_t nv = (int64_t)nx * ny * nz;
  const double cx0 = 0.5 * (nx - 1), cy0 = 0.5 * (ny - 1), cz0 = 0.5 * (nz - 1);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t v0 = (int64_t)chunk * FF_CHUNK;
  for (int64_t v = v0 + threadIdx.x; v < v0 + FF_CHUNK && v < nv; v += FF_T) {
    const int64_t xy = (int64_t)nx * ny;
    const int z = (int)(v / xy);
    const int64_t r = v - (int64_t)z * xy;
    const int y = (int)(r / nx), x = (int)(r - (int64_t)y * nx);
    const double px = (x - cx0) * dx, py = (y - cy0) * dy, pz = (z - cz0) * dz;
    double s, c;
    sincos(k0 * (rx * px + ry * py + rz * pz), &s, &c);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const c128 p = P[q * nv + v];
      const double cq = c * hc[q] - s * hs[q], sq = s * hc[q] + c * hs[q];
      acc[2 * q] += p.x * cq - p.y * sq;
      acc[2 * q + 1] += p.x * sq + p.y * cq;
    }
  }
  block_sum<6>(acc);
  if (threadIdx.x == 0) {
    double* o = part + ((int64_t)dir * nchunk + chunk) * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) o[k] = acc[k];
  }
}

__global__ void __launch_bounds__(FF_T) k_far_final(const double* part, int nchunk, const double* rhat, double dV,
                                                    c128* F) {
  const int dir = blockIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int c = threadIdx.x; c < nchunk; c += FF_T) {
    const double* p = part + ((int64_t)dir * nchunk + c) * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] += p[k];
  }
  block_sum<6>(acc);
  if (threadIdx.x == 0) {
    const double r[3] = {rhat[3 * dir], rhat[3 * dir + 1], rhat[3 * dir + 2]};
    double fr[3], fi[3];
    for (int q = 0; q < 3; ++q) {
      fr[q] = acc[2 * q] * dV;
      fi[q] = acc[2 * q + 1] * dV;
    }
    const double dr = r[0] * fr[0] + r[1] * fr[1] + r[2] * fr[2];
    const double di = r[0] * fi[0] + r[1] * fi[1] + r[2] * fi[2];
    for (int q = 0; q < 3; ++q) F[3 * dir + q] = mk<double>(fr[q] - r[q] * dr, fi[q] - r[q] * di);
  }
}

int64_t far_field_chunks(int64_t nv) { return (nv + FF_CHUNK - 1) / FF_CHUNK; }

int64_t far_field_scratch_doubles() { return kFarScratchDoubles; }

void* far_field_scratch_address() {
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    throw std::runtime_error(std::string("far-field scratch address: ") + hipGetErrorString(e));
  return ptr;
}

void far_field(const c128* P, int nx, int ny, int nz, double dx, double dy, double dz, double k0, const double* rhat,
               int ndir, double* part, c128* F, hipStream_t s, bool faces) {
  if (ndir <= 0) return;
  const int64_t nchunk = far_field_chunks((int64_t)nx * ny * nz);
  hipLaunchKernelGGL(k_far_partial, dim3((unsigned)(ndir * nchunk)), dim3(FF_T), 0, s, P, nx, ny, nz, dx, dy, dz,
                     k0, rhat, (int)nchunk, part, faces ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("far field launch: ") + hipGetErrorString(e));
  hipLaunchKernelGGL(k_far_final, dim3(ndir), dim3(FF_T), 0, s, part, (int)nchunk, rhat, dx * dy * dz, F);
  e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string("far field launch: ") + hipGetErrorString(e));
}

}  // namespace vie
