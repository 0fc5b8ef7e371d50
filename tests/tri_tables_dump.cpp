// Prints the compile-time channel and correlation tables of the TRI vertex
// kernels (csrc/kernels_tri.h), host build, for tests/test_tri_tables.py:
//   T ch i c1 c2 q k     one line per channel term (ch 0..4: s, u, the two
//                        t-channel corrections, the RPA term)
//   X m qp x             one line per correlation exchange coefficient
#include <cstdio>

#include "kernels_tri.h"

int main() {
    for (int ch = 0; ch <= pffrg::kTriRpa; ++ch)
        for (int i = 0; i < 256; ++i) {
            const pffrg::TriTerm t = pffrg::tri_term(ch, i);
            std::printf("T %d %d %d %d %d %d\n", ch, i, t.c1, t.c2, t.q, t.k);
        }
    for (int m = 0; m < 16; ++m)
        for (int qp = 0; qp < 16; ++qp) std::printf("X %d %d %d\n", m, qp, pffrg::tri_chi_x(m, qp));
    return 0;
}
