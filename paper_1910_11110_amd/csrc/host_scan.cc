// host_scan.cc -- host-only scans of submitted chunks (plain C++, no device code).
#include <stdint.h>

namespace vc {

// whether any event of a chunk is malformed (a reserved bit set, an op above Noop, or an
// id at or above n_ids <= 2^24): one branch-free pass that the compiler vectorizes, in
// an AVX2 clone chosen at load time where the host has it
__attribute__((target_clones("avx2", "default"))) bool any_malformed(const uint32_t *ev, uint32_t n, uint32_t n_ids)
{
    uint32_t bad = 0;
    for (uint32_t i = 0; i < n; i++) {
        const uint32_t w = ev[i];
        const int32_t d = (int32_t)(w & 0xFFFFFFu) - (int32_t)n_ids; // >= 0: id out of range
        bad |= (w & 0xF0000000u) | ((((w >> 24) & 7u) + 3u) & 8u) | (~(uint32_t)d >> 31);
    }
    return bad != 0;
}

} // namespace vc
