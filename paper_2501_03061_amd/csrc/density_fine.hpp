// The density on the charge-density grid, twice as fine per axis as the
// wavefunction grid (Sec. VI), for orbitals with occupations (Eq. 12): each
// orbital is Fourier-interpolated onto the fine grid, one axis after the
// other, then rho_f = sum_i occ_i |phi_i^f|^2 in FP64.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace px {

// Orbitals per chunk of the interpolation (its scratch is 10 N_g values per orbital).
constexpr int kFineChunk = 16;

// Workspace bytes of launch_density_fine for grid n[3] (even axes).
size_t density_fine_work_bytes(bool fp32, const int* n, int norb);

// rho_fine [2 n2][2 n1][2 n0] = sum_i occ_i |phi_i^f|^2, phi [norb][N_g]
// (complex64 if fp32 else complex128); work: density_fine_work_bytes.
hipError_t launch_density_fine(bool fp32, const int* n, int norb, const void* phi, const double* occ,
                               double* rho_fine, void* work, hipStream_t s);

}  // namespace px
