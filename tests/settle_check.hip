// Host driver for the exact sign routines of the near-half decision
// (paper_1808_02950_amd/csrc/settle.hpp): reads lines "a b c d p q" (decimal
// integers) and prints the sign of (a + b sqrt p) + (c + d sqrt p) sqrt q as
// the kernels compute it.  Built and run by tests/test_settle_sign.py.
#include <cstdio>
#include <cstring>

#include "settle.hpp"

static adct::i128 parse(const char *s) {
    bool neg = *s == '-';
    if (neg || *s == '+') ++s;
    adct::i128 v = 0;
    for (; *s; ++s) v = v * 10 + (*s - '0');
    return neg ? -v : v;
}

int main() {
    char a[64], b[64], c[64], d[64];
    unsigned p, q;
    while (std::scanf("%63s %63s %63s %63s %u %u", a, b, c, d, &p, &q) == 6)
        std::printf("%d\n", adct::sgn_field(parse(a), parse(b), parse(c), parse(d), p, q));
    return 0;
}
