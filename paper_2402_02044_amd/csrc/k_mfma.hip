// k_mfma.hip -- placeholder until the MFMA scan lands
#include "lvq_internal.h"
namespace lvq {
hipError_t launch_scan_mfma(const ScanArgs &, int, int, hipStream_t) { return hipErrorNotSupported; }
}
