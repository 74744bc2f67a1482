// Host check of the storage layout's index arithmetic (the functions the kernels
// use, compiled for the host): on 3-D levels every grid node maps to its own
// storage index inside the arrays, the index decodes back to the node, and every
// lane of every brick item addresses the node it names; on 2-D levels the index is
// the row layout's.  Exit status 0 when every check holds.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>
#include "lsmg_dev.hpp"
using namespace lsmg;
int main()
{
    int bad = 0;
    for (int n : {5, 9, 17, 33, 65, 129, 257}) {
        const long long half = (n + 1) / 2;
        const int Wp = (int)((half + (1 << kBP) - 1) >> kBP << kBP);
        const long long cs = 32LL * brick_np(Wp) * brick_nj(n) * brick_nk(n), ss = 2 * cs;
        std::vector<char> seen((size_t)ss, 0);
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    const long long q = sidx(3, n, Wp, cs, i, j, k);
                    if (q < 0 || q >= ss) { if (bad++ < 5) printf("range\n"); continue; }
                    if (seen[(size_t)q]) { if (bad++ < 5) printf("dup\n"); }
                    seen[(size_t)q] = 1;
                    int a, b, c;
                    sidx_node<3>(n, Wp, cs, q, a, b, c);
                    if (a != i || b != j || c != k) { if (bad++ < 5) printf("decode\n"); }
                }
        const int np = brick_np(Wp), nj = brick_nj(n), nk = brick_nk(n);
        for (int col = 0; col < 2; ++col)
            for (int kb = 0; kb < nk; ++kb)
                for (int jb = 0; jb < nj; ++jb)
                    for (int pb = 0; pb < np; pb += 2) {
                        int4 w = make_int4(col, pb | (jb << 10) | (kb << 20), -1, -1);
                        for (int lane = 0; lane < 64; ++lane) {
                            if ((lane >> 5) && pb + 1 >= np) continue;
                            long long idx; int i, j, k;
                            brick_lane(n, Wp, cs, col, w, lane, idx, i, j, k);
                            if (idx < 0 || idx >= ss) { if (bad++ < 5) printf("lane idx range\n"); continue; }
                            if (i < n && j < n && k < n && sidx(3, n, Wp, cs, i, j, k) != idx) { if (bad++ < 5) printf("lane mismatch\n"); }
                        }
                    }
    }
    // 2-D: colour-split rows
    for (int n : {9, 65, 1025}) {
        const int Wp = ((n + 1) / 2 + 15) / 16 * 16;
        const long long cs = (long long)n * Wp;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const long long q = ((i + j) & 1) * cs + (long long)j * Wp + (i >> 1);
                if (sidx(2, n, Wp, cs, i, j, 0) != q) { if (bad++ < 5) printf("2-D index\n"); }
                int a, b, c;
                sidx_node<2>(n, Wp, cs, q, a, b, c);
                if (a != i || b != j || c != 0) { if (bad++ < 5) printf("2-D decode\n"); }
            }
    }
    printf("brick %dx%dx%d (positions x rows x planes): %d failures\n", 1 << kBP, 1 << kBJ, 1 << kBK, bad);
    return bad != 0;
}
