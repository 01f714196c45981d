// transport.hip -- radial and vertical transport of every active particle
// (paper, Summary), the end-of-step bookkeeping and a Philox test kernel.
//
// Per particle, at its own (r, z): local gas of the power-law disk, Stokes
// number, turbulent diffusivity D = alpha c_s H / (1 + St^2); a random walk
// with uniform kicks of variance 2 D dt; settling toward the midplane and
// the gas-density correction D/H^2 taken semi-implicitly; radial drift plus
// the diffusion drift (D/r) d ln(r Sigma_g D)/d ln r (5/2 - q - p for the
// power-law disk), under which the axisymmetric walk keeps tracers
// distributed like the gas; |z| folded by mirror symmetry; particles inside
// r_in leave the grid.  One thread per particle,
// coalesced FP64 loads and stores.
#include "device_common.hpp"
#include "internal.hpp"

namespace mcd {

__global__ __launch_bounds__(256) void transport_kernel(Model P, double *__restrict__ r,
                                                        double *__restrict__ z,
                                                        const double *__restrict__ m,
                                                        uint8_t *__restrict__ active, int64_t N,
                                                        double dt, const DevState *st) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N || !active[k]) return;
  const uint32_t step = st->step;
  const double rk = P.column ? P.r_col : r[k];
  const double zk = z[k];
  const LocalGas d = local_gas_at(P, rk, zk);
  const double v_th = sqrt(8.0 / kPi) * d.cs;
  const double lambda = P.mu * kMassH / (d.rho_g * kSigmaH2);
  const double nu = 0.5 * v_th * lambda;
  const double a = cbrt(3.0 * m[k] / (4.0 * kPi * P.rho_s));
  const double St = stopping_time(P.rho_s, a, d.rho_g, v_th, lambda, nu) * d.Omega;
  const double D = d.alpha * d.cs * d.H / (1.0 + St * St);
  const U4 w = philox4x32_10(U4{(uint32_t)k, 0u, step, 2u}, P.key0, P.key1);
  const double kick_r = 2.0 * u01(w.x, w.y) - 1.0;
  const double kick_z = 2.0 * u01(w.z, w.w) - 1.0;

  double kz = 0.0, dz = 0.0;
  if (P.flags & TR_SETTLE) kz += d.Omega * St / (1.0 + St);
  if (P.flags & TR_MIX_Z) {
    kz += D / (d.H * d.H);
    dz = kick_z * sqrt(6.0 * D * dt);
  }
  z[k] = fabs((zk + dz) / (1.0 + kz * dt));

  if (!P.column) {
    double v = 0.0, dr = 0.0;
    if (P.flags & TR_DRIFT) {
      const double eta_vK = 0.5 * d.cs * d.cs / (d.Omega * rk) * d.slopeP;
      v += -2.0 * eta_vK * St / (1.0 + St * St);
    }
    if (P.flags & TR_MIX_R) {
      v += D * d.corr / rk;
      dr = kick_r * sqrt(6.0 * D * dt);
    }
    const double rn = rk + v * dt + dr;
    r[k] = rn;
    if (rn < P.r_in) active[k] = 0;
  }
}

__global__ void finish_step(DevState *st, double dt) {
  st->step += 1u;
  st->t_sim += dt;
}

__global__ void philox_kernel(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out,
                              int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const U4 c{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
  const U4 o = philox4x32_10(c, k0, k1);
  out[4 * i] = o.x;
  out[4 * i + 1] = o.y;
  out[4 * i + 2] = o.z;
  out[4 * i + 3] = o.w;
}

hipError_t launch_transport(const Model &P, double *r, double *z, const double *m,
                            uint8_t *active, int64_t N, double dt, DevState *state,
                            hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const int64_t blocks = (N + 255) / 256;
  transport_kernel<<<(unsigned)blocks, 256, 0, s>>>(P, r, z, m, active, N, dt, state);
  return hipGetLastError();
}

hipError_t launch_finish_step(DevState *state, double dt, hipStream_t s) {
  finish_step<<<1, 1, 0, s>>>(state, dt);
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out, int64_t n,
                         hipStream_t s) {
  if (n <= 0) return hipSuccess;
  philox_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ctr, k0, k1, out, n);
  return hipGetLastError();
}

}  // namespace mcd
