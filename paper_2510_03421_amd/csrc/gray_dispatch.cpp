// Routes a Gray-walk launch (engine or e_m form) to the translation unit that
// instantiates its vector length.
#include "esym_band_ranges.h"
#include "internal.h"

namespace permgpu {

int gray_occ_real_a(int nv);
hipError_t gray_launch_real_a(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
int gray_occ_real_b(int nv);
hipError_t gray_launch_real_b(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
int gray_occ_real_c(int nv);
hipError_t gray_launch_real_c(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
int gray_occ_real_pair(int nv);
hipError_t gray_launch_real_pair(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
int gray_occ_cplx_a(int nv);
hipError_t gray_launch_cplx_a(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
int gray_occ_cplx_b(int nv);
hipError_t gray_launch_cplx_b(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
int gray_occ_cplx_c(int nv);
hipError_t gray_launch_cplx_c(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
int gray_occ_int_a(int nv);
hipError_t gray_launch_int_a(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
int gray_occ_int_b(int nv);
hipError_t gray_launch_int_b(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
int gray_occ_int_c(int nv);
hipError_t gray_launch_int_c(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
int gray_occ_int_d(int nv);
hipError_t gray_launch_int_d(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);

int gray_engine_blocks_per_cu_real(int nv) {
  if (nv >= 1 && nv <= 24) return gray_occ_real_a(nv);
  if (nv >= 25 && nv <= 40) return gray_occ_real_b(nv);
  if (nv >= 41 && nv <= 48) return gray_occ_real_c(nv);
  return 0;
}

hipError_t launch_gray_engine_real(const GrayWalk &w, int grid, int block, void *partials,
                                   hipStream_t s) {
  if (w.nv >= 1 && w.nv <= 24) return gray_launch_real_a(w, grid, block, partials, s);
  if (w.nv >= 25 && w.nv <= 40) return gray_launch_real_b(w, grid, block, partials, s);
  if (w.nv >= 41 && w.nv <= 48) return gray_launch_real_c(w, grid, block, partials, s);
  return hipErrorInvalidValue;
}

int gray_engine_blocks_per_cu_real_pair(int nv) {
  if (nv >= GRAY_PAIR_MIN_NV && nv <= GRAY_PAIR_MAX_NV) return gray_occ_real_pair(nv);
  return 0;
}

hipError_t launch_gray_engine_real_pair(const GrayWalk &w, int grid, int block, void *partials,
                                        hipStream_t s) {
  if (w.nv >= GRAY_PAIR_MIN_NV && w.nv <= GRAY_PAIR_MAX_NV && !w.wlist && w.b >= 3 &&
      w.blocks_per_lane % 4 == 0)
    return gray_launch_real_pair(w, grid, block, partials, s);
  return hipErrorInvalidValue;
}

int gray_engine_blocks_per_cu_cplx(int nv) {
  if (nv >= 1 && nv <= 24) return gray_occ_cplx_a(nv);
  if (nv >= 25 && nv <= 40) return gray_occ_cplx_b(nv);
  if (nv >= 41 && nv <= 48) return gray_occ_cplx_c(nv);
  return 0;
}

hipError_t launch_gray_engine_cplx(const GrayWalk &w, int grid, int block, void *partials,
                                   hipStream_t s) {
  if (w.nv >= 1 && w.nv <= 24) return gray_launch_cplx_a(w, grid, block, partials, s);
  if (w.nv >= 25 && w.nv <= 40) return gray_launch_cplx_b(w, grid, block, partials, s);
  if (w.nv >= 41 && w.nv <= 48) return gray_launch_cplx_c(w, grid, block, partials, s);
  return hipErrorInvalidValue;
}

int gray_engine_blocks_per_cu_int(int nv) {
  if (nv >= 1 && nv <= 16) return gray_occ_int_a(nv);
  if (nv >= 17 && nv <= 26) return gray_occ_int_b(nv);
  if (nv >= 27 && nv <= 34) return gray_occ_int_c(nv);
  if (nv >= 35 && nv <= 40) return gray_occ_int_d(nv);
  return 0;
}

hipError_t launch_gray_engine_int(const GrayWalk &w, int grid, int block, void *partials,
                                   hipStream_t s) {
  if (w.nv >= 1 && w.nv <= 16) return gray_launch_int_a(w, grid, block, partials, s);
  if (w.nv >= 17 && w.nv <= 26) return gray_launch_int_b(w, grid, block, partials, s);
  if (w.nv >= 27 && w.nv <= 34) return gray_launch_int_c(w, grid, block, partials, s);
  if (w.nv >= 35 && w.nv <= 40) return gray_launch_int_d(w, grid, block, partials, s);
  return hipErrorInvalidValue;
}

int esym_occ_real_a(int nv);
int esym_occ_real_b(int nv);
int esym_occ_cplx_a(int nv);
int esym_occ_cplx_b(int nv);
hipError_t esym_launch_real_a(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
hipError_t esym_launch_real_b(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
hipError_t esym_launch_cplx_a(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
hipError_t esym_launch_cplx_b(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);

int esym_occ_int_a(int nv);
int esym_occ_int_b(int nv);
int esym_occ_int_c(int nv);
int esym_occ_int_d(int nv);
int esym_occ_int_e(int nv);
hipError_t esym_launch_int_a(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
hipError_t esym_launch_int_b(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
hipError_t esym_launch_int_c(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
hipError_t esym_launch_int_d(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);
hipError_t esym_launch_int_e(const GrayWalk &w, int grid, int block, void *partials, hipStream_t s);

int esym_blocks_per_cu_int(int nv) {
  if (nv >= 1 && nv <= 24) return esym_occ_int_a(nv);
  if (nv >= 25 && nv <= 32) return esym_occ_int_b(nv);
  if (nv >= 33 && nv <= 40) return esym_occ_int_c(nv);
  if (nv >= 41 && nv <= 44) return esym_occ_int_d(nv);
  if (nv >= 45 && nv <= 48) return esym_occ_int_e(nv);
  return 0;
}
hipError_t launch_esym_int(const GrayWalk &w, int grid, int block, void *partials,
                           hipStream_t s) {
  if (w.nv >= 1 && w.nv <= 24) return esym_launch_int_a(w, grid, block, partials, s);
  if (w.nv >= 25 && w.nv <= 32) return esym_launch_int_b(w, grid, block, partials, s);
  if (w.nv >= 33 && w.nv <= 40) return esym_launch_int_c(w, grid, block, partials, s);
  if (w.nv >= 41 && w.nv <= 44) return esym_launch_int_d(w, grid, block, partials, s);
  if (w.nv >= 45 && w.nv <= 48) return esym_launch_int_e(w, grid, block, partials, s);
  return hipErrorInvalidValue;
}

#define ESYM_BAND_DECL(k, lo, hi)                                                    \
  int esym_band_occ_##k##_##lo(int nv, int m);                                       \
  hipError_t esym_band_launch_##k##_##lo(const GrayWalk &w, int grid, int block,     \
                                         void *partials, hipStream_t s);
ESYM_BAND_RANGES(ESYM_BAND_DECL)
#undef ESYM_BAND_DECL

int esym_band_blocks_per_cu(int kind, int nv, int m) {
  if (m < ESYM_BAND_MIN_M || m > nv || nv > ESYM_BAND_MAX_N) return 0;
#define ESYM_BAND_OCC(k, lo, hi) \
  if (kind == k && m >= lo && m <= hi) return esym_band_occ_##k##_##lo(nv, m);
  ESYM_BAND_RANGES(ESYM_BAND_OCC)
#undef ESYM_BAND_OCC
  return 0;
}

hipError_t launch_esym_band(int kind, const GrayWalk &w, int grid, int block, void *partials,
                            hipStream_t s) {
#define ESYM_BAND_LAUNCH(k, lo, hi) \
  if (kind == k && w.m >= lo && w.m <= hi) return esym_band_launch_##k##_##lo(w, grid, block, partials, s);
  ESYM_BAND_RANGES(ESYM_BAND_LAUNCH)
#undef ESYM_BAND_LAUNCH
  return hipErrorInvalidValue;
}

int esym_blocks_per_cu_real(int nv) {
  if (nv >= 1 && nv <= 24) return esym_occ_real_a(nv);
  if (nv >= 25 && nv <= 48) return esym_occ_real_b(nv);
  return 0;
}
int esym_blocks_per_cu_cplx(int nv) {
  if (nv >= 1 && nv <= 24) return esym_occ_cplx_a(nv);
  if (nv >= 25 && nv <= 48) return esym_occ_cplx_b(nv);
  return 0;
}
hipError_t launch_esym_real(const GrayWalk &w, int grid, int block, void *partials,
                            hipStream_t s) {
  if (w.nv >= 1 && w.nv <= 24) return esym_launch_real_a(w, grid, block, partials, s);
  if (w.nv >= 25 && w.nv <= 48) return esym_launch_real_b(w, grid, block, partials, s);
  return hipErrorInvalidValue;
}
hipError_t launch_esym_cplx(const GrayWalk &w, int grid, int block, void *partials,
                            hipStream_t s) {
  if (w.nv >= 1 && w.nv <= 24) return esym_launch_cplx_a(w, grid, block, partials, s);
  if (w.nv >= 25 && w.nv <= 48) return esym_launch_cplx_b(w, grid, block, partials, s);
  return hipErrorInvalidValue;
}

}  // namespace permgpu
