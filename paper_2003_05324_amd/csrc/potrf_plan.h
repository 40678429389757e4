// Host-side plan of the blocked factorization of one diagonal tile of 256 or 512 columns
// (dpotrf of Algorithm 1, with the tile's inverse): the sequence of launches, each either the
// single-workgroup factorization of one 128 x 128 diagonal block or a set of independent block
// products.  Used by the launcher in potrf.hip and checked on the host by
// tests/potrf_plan_check.cpp (bounds of every product, job counts, and the plan's arithmetic
// replayed in double precision against a plain Cholesky factor and inverse).
//
//   for each block column kb:  L_kk, L_kk^-1 <- factorization of the diagonal block;
//                              X_i = A_ik L_kk^-T for the blocks below it (into scratch);
//                              A_ij -= X_i X_j^T for the trailing blocks, A_ik <- X_i;
//   then the inverse by halves, [[L11, 0], [L21, L22]]^-1 = [[B11, 0], [-B22 L21 B11, B22]]:
//   inside each 256-column half, then (512 columns) between the halves; then the strictly upper
//   blocks of the inverse, used as scratch, are zeroed and the FP32 copy of the inverse written.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

namespace mpgeo {

constexpr int kPotrfBlock = 128;   // block columns of the blocked factorization
constexpr int kPotrfMaxJobs = 8;   // products per launch

enum PotrfBuf { kBufNone = -1, kBufA = 0, kBufB = 1 };   // the tile (A -> L) and its inverse (B)

// C (m x n) <- beta C + alpha A op(B) with op(B) = B^T (B n x k, transb) or B (k x n) when
// k > 0; C <- A when k == 0 and A is given; C <- 0 when it is not.  Offsets in elements of the
// column-major nbp x nbp buffers; m, n multiples of 64 and k of 16.  lower: entries above C's
// diagonal are left untouched.  to32: the FP32 copy of B receives the result too.
struct PotrfJob {
    int c_buf;
    int64_t c_off;
    int a_buf;
    int64_t a_off;
    int b_buf;
    int64_t b_off;
    int m, n, k;
    bool transb, lower, to32;
    double alpha, beta;
};

// diag >= 0: factor diagonal block diag (one workgroup); otherwise one launch of `jobs`.
struct PotrfStep {
    int diag = -1;
    std::vector<PotrfJob> jobs;
};

inline std::vector<PotrfStep> potrf_blocked_plan(int nbp, bool with32) {
    const int P = kPotrfBlock, q = nbp / P;
    auto off = [&](int bi, int bj) { return (int64_t)bi * P + (int64_t)bj * P * nbp; };
    std::vector<PotrfStep> plan;
    std::vector<PotrfJob> cur;
    auto flush = [&] {
        if (!cur.empty()) {
            PotrfStep st;
            st.jobs = cur;
            plan.push_back(st);
            cur.clear();
        }
    };
    auto job = [&](int cb, int64_t co, int ab, int64_t ao, int bb, int64_t bo, int m, int n, int k, bool transb,
                   double alpha, double beta, bool lower = false, bool to32 = false) {
        if ((int)cur.size() == kPotrfMaxJobs) flush();
        cur.push_back(PotrfJob{cb, co, ab, ao, bb, bo, m, n, k, transb, lower, to32, alpha, beta});
    };
    for (int kb = 0; kb < q; ++kb) {
        PotrfStep d;
        d.diag = kb;
        plan.push_back(d);
        if (kb + 1 == q) break;
        for (int i = kb + 1; i < q; ++i)   // X_i into the scratch block (kb, i)
            job(kBufB, off(kb, i), kBufA, off(i, kb), kBufB, off(kb, kb), P, P, P, true, 1.0, 0.0);
        flush();
        for (int j = kb + 1; j < q; ++j)
            for (int i = j; i < q; ++i)
                job(kBufA, off(i, j), kBufB, off(kb, i), kBufB, off(kb, j), P, P, P, true, -1.0, 1.0, i == j);
        for (int i = kb + 1; i < q; ++i) job(kBufA, off(i, kb), kBufB, off(kb, i), kBufNone, 0, P, P, 0, false, 1.0, 0.0);
        flush();
    }
    // inverse inside each 256-column half; T = L_{h+1,h} B_hh in a strictly upper block
    std::vector<int64_t> tpos;
    for (int h = 0; h + 1 < q; h += 2) {
        tpos.push_back((h + 2 < q) ? off(h, h + 2) : off(0, 1));
        job(kBufB, tpos.back(), kBufA, off(h + 1, h), kBufB, off(h, h), P, P, P, false, 1.0, 0.0);
    }
    flush();
    for (int h = 0, t = 0; h + 1 < q; h += 2, ++t)
        job(kBufB, off(h + 1, h), kBufB, off(h + 1, h + 1), kBufB, tpos[(size_t)t], P, P, P, false, -1.0, 0.0);
    flush();
    if (q == 4) {   // between the halves: B(2:3, 0:1) = -B(2:3, 2:3) (L(2:3, 0:1) B(0:1, 0:1))
        job(kBufB, off(0, 1), kBufNone, 0, kBufNone, 0, P, P, 0, false, 0.0, 0.0);   // B(0:1, 0:1)'s upper block
        job(kBufB, off(2, 3), kBufNone, 0, kBufNone, 0, P, P, 0, false, 0.0, 0.0);   // B(2:3, 2:3)'s upper block
        flush();
        job(kBufB, off(0, 2), kBufA, off(2, 0), kBufB, off(0, 0), 2 * P, 2 * P, 2 * P, false, 1.0, 0.0);
        flush();
        job(kBufB, off(2, 0), kBufB, off(2, 2), kBufB, off(0, 2), 2 * P, 2 * P, 2 * P, false, -1.0, 0.0);
        flush();
    }
    // strictly upper blocks to zero; the FP32 copy of every block
    for (int j = 0; j < q; ++j)
        for (int i = 0; i < q; ++i) {
            if (i < j) job(kBufB, off(i, j), kBufNone, 0, kBufNone, 0, P, P, 0, false, 0.0, 0.0, false, with32);
            else if (with32) job(kBufB, off(i, j), kBufB, off(i, j), kBufNone, 0, P, P, 0, false, 1.0, 0.0, false, true);
        }
    flush();
    return plan;
}

}  // namespace mpgeo
