// gks_inst.hip -- explicit instantiations of the face kernels, one share per compilation.
//
// The build compiles this unit once for each GKS_PART (0..7), so that the flux kernels,
// which take most of the compile time, are compiled in parallel.  Every share defines
// kernels that gks_kernels.hpp declares `extern template`; together the shares cover
// GKS_TILE2_VARIANTS, GKS_TILE3_VARIANTS and GKS_FACE_VARIANTS exactly once.
#include "gks_kernels.hpp"

#ifndef GKS_PART
#error "compile with -DGKS_PART=<0..7>"
#endif

namespace gks {

#define GKS_TILE2_D(V) template __global__ void k_tile2<double, V, 0>(const void*, int, int);
#define GKS_TILE2_F(V) template __global__ void k_tile2<float, V, 0>(const void*, int, int);
#define GKS_FACE_D(T, V) template __global__ void k_face<double, 3, T, V>(const void*, int, int);
#define GKS_FACE_F(T, V) template __global__ void k_face<float, 3, T, V>(const void*, int, int);
#define GKS_TILE3_D(V) template __global__ void k_tile3<double, V>(const void*, int, int);
#define GKS_TILE3_F(V) template __global__ void k_tile3<float, V>(const void*, int, int);

// 2D tiles: MUSCL reconstructions with transport and tau_hat (variants 0..7), then the
// multi-dimensional expansion and WENO5 (8..11, 16..19)
#if GKS_PART == 0
GKS_TILE2_D(0) GKS_TILE2_D(1) GKS_TILE2_D(2) GKS_TILE2_D(3) GKS_TILE2_D(4) GKS_TILE2_D(5) GKS_TILE2_D(6) GKS_TILE2_D(7)
#elif GKS_PART == 1
GKS_TILE2_D(8) GKS_TILE2_D(9) GKS_TILE2_D(10) GKS_TILE2_D(11)
GKS_TILE2_D(16) GKS_TILE2_D(17) GKS_TILE2_D(18) GKS_TILE2_D(19)
#elif GKS_PART == 2
GKS_TILE2_F(0) GKS_TILE2_F(1) GKS_TILE2_F(2) GKS_TILE2_F(3) GKS_TILE2_F(4) GKS_TILE2_F(5) GKS_TILE2_F(6) GKS_TILE2_F(7)
#elif GKS_PART == 3
GKS_TILE2_F(8) GKS_TILE2_F(9) GKS_TILE2_F(10) GKS_TILE2_F(11)
GKS_TILE2_F(16) GKS_TILE2_F(17) GKS_TILE2_F(18) GKS_TILE2_F(19)
// 3D: the fused tile kernel (the plain scheme, tau_hat, third-order MUSCL, each with
// frozen or transported k and omega) and the face kernel of the multi-dimensional expansion
// and WENO5
#elif GKS_PART == 4
GKS_TILE3_D(0) GKS_TILE3_D(2) GKS_TILE3_D(4) GKS_TILE3_D(6)
GKS_TILE3_D(1) GKS_TILE3_D(3) GKS_TILE3_D(5) GKS_TILE3_D(7)
template __global__ void k_tile2<double, 0, 1>(const void*, int, int);
#elif GKS_PART == 5
template __global__ void k_tile2<double, 0, 2>(const void*, int, int);
GKS_FACE_D(64, 8) GKS_FACE_D(64, 9) GKS_FACE_D(64, 10) GKS_FACE_D(64, 11)
GKS_FACE_D(64, 16) GKS_FACE_D(64, 17) GKS_FACE_D(64, 18) GKS_FACE_D(64, 19)
#elif GKS_PART == 6
GKS_TILE3_F(0) GKS_TILE3_F(2) GKS_TILE3_F(4) GKS_TILE3_F(6)
GKS_TILE3_F(1) GKS_TILE3_F(3) GKS_TILE3_F(5) GKS_TILE3_F(7)
template __global__ void k_tile2<float, 0, 1>(const void*, int, int);
#elif GKS_PART == 7
template __global__ void k_tile2<float, 0, 2>(const void*, int, int);
GKS_FACE_F(64, 8) GKS_FACE_F(64, 9) GKS_FACE_F(64, 10) GKS_FACE_F(64, 11)
GKS_FACE_F(64, 16) GKS_FACE_F(64, 17) GKS_FACE_F(64, 18) GKS_FACE_F(64, 19)
#else
#error "GKS_PART out of range"
#endif

}  // namespace gks
