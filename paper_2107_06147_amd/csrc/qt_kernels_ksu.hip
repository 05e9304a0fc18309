// qt_kernels_ksu.hip -- the fused persistent kernel instantiated for the
// isotropic KSU potential (appendix "Isotropic KSU potential"): one block
// size per (precision, N), compiled apart from the Munich variants so that
// each keeps its own register allocation.
#include "qt_fused.hpp"

namespace qt {

#define QT_K32(N, W) {QT_FP32_BULK, N, W, launch_fused<float, N, W, QT_POTENTIAL_KSU>, \
                      occupancy_fused<float, N, W, QT_POTENTIAL_KSU>}
#define QT_K64(N, W) {QT_FP64, N, W, launch_fused<double, N, W, QT_POTENTIAL_KSU>, \
                      occupancy_fused<double, N, W, QT_POTENTIAL_KSU>}

static const FusedEntry kFusedKsu[] = {
    QT_K32(256, 64),  QT_K32(512, 64),  QT_K32(1024, 128), QT_K32(2048, 256),
    QT_K32(4096, 512), QT_K32(8192, 1024),
    QT_K64(256, 64),  QT_K64(512, 128), QT_K64(1024, 256), QT_K64(2048, 512),
    QT_K64(4096, 1024), QT_K64(8192, 1024),
};

bool fused_ksu_variant(int prec, int N, int* W, fused_launcher* launch, int* slots_per_cu)
{
    for (const auto& e : kFusedKsu)
        if (e.prec == prec && e.N == N) {
            *W = e.W;
            *launch = e.launch;
            *slots_per_cu = e.occ();
            return true;
        }
    return false;
}

}  // namespace qt
