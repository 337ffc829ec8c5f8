// Reference Philox4x32-10 words from rocRAND's own engine (host side of its
// header API), used only by the tests to pin the oracle's and the library's
// independent Philox implementations.  rocRAND maps a counter (c0, c1, c2, c3)
// to offset = 4 (c0 + 2^32 c1) numbers into subsequence c2 + 2^32 c3.
#include <rocrand/rocrand_kernel.h>

extern "C" void ref_philox4x32_10(unsigned long long seed, const unsigned int *ctr,
                                  unsigned int *out) {
    rocrand_state_philox4x32_10 st;
    const unsigned long long offset =
        4ull * ((unsigned long long)ctr[0] | ((unsigned long long)ctr[1] << 32));
    const unsigned long long subseq =
        (unsigned long long)ctr[2] | ((unsigned long long)ctr[3] << 32);
    rocrand_init(seed, subseq, offset, &st);
    const uint4 r = rocrand4(&st);
    out[0] = r.x;
    out[1] = r.y;
    out[2] = r.z;
    out[3] = r.w;
}
