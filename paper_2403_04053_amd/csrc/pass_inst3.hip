// Pencil-pass kernels of the tile shapes assigned to compilation unit 3
// (pass_variants.hpp).
#include "pass_kernel.hpp"
#include "pass_variants.hpp"

namespace pstd {

#define PSTD_UNIT_0(N_, A_, B_, M_, P_, S_)
#define PSTD_UNIT_1(N_, A_, B_, M_, P_, S_)
#define PSTD_UNIT_2(N_, A_, B_, M_, P_, S_)
#define PSTD_UNIT_3(N_, A_, B_, M_, P_, S_) PSTD_DEFINE_SHAPE(N_, A_, B_, M_, P_, S_)
#define PSTD_UNIT_4(N_, A_, B_, M_, P_, S_)
#define PSTD_UNIT_5(N_, A_, B_, M_, P_, S_)
#define PSTD_SELECT(N_, A_, B_, M_, P_, S_, PART_) PSTD_UNIT_##PART_(N_, A_, B_, M_, P_, S_)
PSTD_VARIANTS(PSTD_SELECT)

}  // namespace pstd
