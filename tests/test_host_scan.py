"""Host code of the serving path: the vectorized scan that refuses a malformed chunk at
submission agrees with the per-event rule (reserved bits 28-31 clear, op at most Noop,
id below n_ids) on every word class, including the ids next to n_ids and ops 4 to 7."""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "..", "paper_1910_11110_amd", "csrc", "host_scan.cc")

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
namespace vc { bool any_malformed(const uint32_t *ev, uint32_t n, uint32_t n_ids); }
static bool bad_word(uint32_t w, uint32_t n_ids)
{
    return (w >> 28) != 0 || ((w >> 24) & 7u) > 4 || (w & 0xFFFFFFu) >= n_ids;
}
int main()
{
    uint64_t x = 88172645463325252ull;
    auto next = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
    const uint32_t ids[] = {1, 2, 63, 64, 5000, 1u << 20, (1u << 24) - 1, 1u << 24};
    long fails = 0, checked = 0;
    uint32_t buf[67];
    for (uint32_t n_ids : ids)
        for (int k = 0; k < 100000; k++) {
            const uint64_t r = next();
            // a candidate word: id near n_ids or anywhere, any op and side, reserved bits
            // set one time in eight
            uint32_t id = (r & 1) ? (uint32_t)((n_ids + (uint32_t)((r >> 1) & 7u)) - 4u) : (uint32_t)((r >> 8) % n_ids);
            id &= 0xFFFFFFu;
            uint32_t w = id | (uint32_t)((r >> 32) & 7u) << 24 | (uint32_t)((r >> 35) & 1u) << 27;
            if (((r >> 40) & 7u) == 0)
                w |= 1u << (28 + ((r >> 43) & 3u));
            // in a chunk of well-formed words, at a random place, chunk lengths 1..67
            const uint32_t n = 1 + (uint32_t)((r >> 48) % 67), at = (uint32_t)((r >> 56) % n);
            for (uint32_t i = 0; i < n; i++)
                buf[i] = (uint32_t)(next() % n_ids) | (uint32_t)(i % 5) << 24;
            buf[at] = w;
            checked++;
            if (vc::any_malformed(buf, n, n_ids) != bad_word(w, n_ids))
                fails++;
        }
    // empty chunk
    if (vc::any_malformed(buf, 0, 1))
        fails++;
    printf("%ld of %ld\n", fails, checked);
    return fails != 0;
}
"""


def test_vectorized_scan_matches_per_event_rule():
    with tempfile.TemporaryDirectory() as d:
        drv = os.path.join(d, "drv.cc")
        exe = os.path.join(d, "drv")
        open(drv, "w").write(DRIVER)
        subprocess.check_call(["g++", "-O3", "-std=c++17", SRC, drv, "-o", exe])
        r = subprocess.run([exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr
