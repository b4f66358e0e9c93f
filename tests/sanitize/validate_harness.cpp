// Runs the host-side argument checks of the C ABI (lfbp_validate.cpp) under
// AddressSanitizer and UndefinedBehaviorSanitizer (built by
// tests/test_sanitizers.py with g++) on ordinary, degenerate and extreme
// shapes: no check overflows or reads out of bounds, and a few outcomes are
// pinned.  Exit status 0 on success.
#include <cstdint>
#include <cstdio>
#include <limits>

#include "lfbp_validate.h"

using namespace lfbp;

namespace {

uint64_t state = 0x9E3779B97F4A7C15ull;
uint64_t next_u64()
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
}

int64_t pick_dim()
{
    static const int64_t special[] = {-1, 0, 1, 2, 3, 15, 165, 2047, 2049, 65535, 1 << 20, int64_t(1) << 31,
                                      int64_t(1) << 40, std::numeric_limits<int64_t>::max()};
    const uint64_t r = next_u64();
    if (r % 3 == 0) return special[(r >> 8) % (sizeof(special) / sizeof(special[0]))];
    return int64_t((r >> 8) % 4097) | 1;
}

int expect(bool ok, const char* what)
{
    if (!ok) std::fprintf(stderr, "unexpected outcome: %s\n", what);
    return ok ? 0 : 1;
}

}  // namespace

int main()
{
    int bad = 0;
    const float* P = reinterpret_cast<const float*>(uintptr_t(1) << 40);   // never dereferenced
    const float* Q = reinterpret_cast<const float*>(uintptr_t(1) << 44);
    float* O = reinterpret_cast<float*>(uintptr_t(1) << 46);
    for (int i = 0; i < 200000; ++i) {
        const lfbp_shape s{pick_dim(), pick_dim(), pick_dim(), pick_dim(), pick_dim()};
        const int64_t R = pick_dim(), C = pick_dim();
        const lfbp_dtype dt = (i & 1) ? LFBP_F16 : LFBP_F32;
        (void)check_shape(s, (i & 1) ? 2 : 4);
        (void)check_gather(P, O, s, dt);
        (void)check_project_shape(s, R, C, unsigned(i % 8));
        (void)check_project(P, s, Q, R, C, O, (i & 2) != 0);
        (void)check_rl(P, Q, s, Q, R, C, Q, Q, O);
        (void)check_grad_psf(P, Q, s, R, C, O);
        (void)ranges_overlap(P, uint64_t(next_u64()), O, uint64_t(next_u64()));
        (void)shape_elems(s);
    }
    const lfbp_shape ok{165, 165, 15, 15, 21}, even{164, 165, 15, 15, 21}, zero{165, 165, 15, 0, 21};
    bad |= expect(check_shape(ok, 4) == LFBP_OK, "microscope shape");
    bad |= expect(check_shape(even, 4) == LFBP_ESHAPE, "even ns");
    bad |= expect(check_shape(zero, 4) == LFBP_ESHAPE, "zero ny");
    bad |= expect(check_project_shape(ok, 600, 600, kProjFwd | kProjBwd | kProjGrad) == LFBP_OK, "projector workload");
    bad |= expect(check_project_shape(ok, 0, 600, kProjFwd) == LFBP_EINVAL, "R = 0");
    bad |= expect(check_gather(P, P, ok, LFBP_F32) == LFBP_EALIAS, "H == Ht");
    bad |= expect(check_gather(nullptr, O, ok, LFBP_F32) == LFBP_EINVAL, "null H");
    if (!bad) std::printf("validate harness: all checks passed\n");
    return bad;
}
