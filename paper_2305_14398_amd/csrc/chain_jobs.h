// The grouped-launch jobs one circuit contributes at chain iteration j
// (stage 4 expansion of step j and, for j >= 1, the j-th product of
// Algorithm 1), given the circuit's buffers.  Shared by batch plans and the
// serving engine so both follow the same buffer discipline as
// qsim_unitary_chain:
//   float32: U_1 is expanded row-major into X[(k-1)%2]; product j reads the
//            column-major step operator S and X[(k-j)%2], writes X[(k-1-j)%2];
//            the last product lands in X[0] = d_U.
//   split:   U_1 is expanded column-major in split form into P[0]; product j
//            (j < k-1) writes (S U)^T in split form to the other P buffer; the
//            last product is taken in the direct orientation into float32 d_U.
#pragma once

#include <cstring>
#include <vector>

#include "host.h"

namespace qsim {

struct ChainCursor {
    int n = 0, k = 0, prec = 0, cfg = 0;
    const qsim_gate* gates = nullptr;
    std::vector<int32_t> off;  // k+1 step offsets
    void* U = nullptr;         // final row-major float32 output
    void* S = nullptr;         // step operator scratch
    void* W1 = nullptr;        // float32: second ping-pong buffer; split: P[0]
    void* W2 = nullptr;        // split: P[1]
    int cur = 0;               // split: index of the P buffer holding the running product

    static int expand_blocks(int n) {
        const long long items = (1ll << (2 * n)) >> 2;
        const long long b = (items + 255) / 256;
        return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
    }
    static int tiles_of(int n, int cfg) {
        if (cfg == 0) return 1;
        const int t = (1 << n) / cfg;
        return t * t;
    }

    // Fills the expansion job of iteration j and, for j >= 1, the product job
    // (returns whether a product job was produced).  Must be called for
    // j = 0, 1, ..., max(k, 1) - 1 in order.
    qsim_status emit(int j, ExpandJob& E, GemmJob& Gj, bool& has_gemm) {
        std::memset(&E, 0, sizeof E);
        has_gemm = false;
        const bool split = is_split(prec);
        const OpFormat fmt = format_of(prec);
        E.n = n;
        E.blocks = expand_blocks(n);
        if (k == 0) {  // the identity
            E.out = U;
            E.fmt = FMT_F32;
            return make_step(n, nullptr, 0, E.st);
        }
        qsim_status s = make_step(n, gates + off[j], off[j + 1] - off[j], E.st);
        if (s != QSIM_OK) return s;
        void* X[2] = {U, W1};
        void* P[2] = {W1, W2};
        if (j == 0) {
            if (!split || k == 1) {
                E.out = split ? U : X[(k - 1) & 1];
                E.fmt = FMT_F32;
                E.layout_col = 0;
            } else {
                E.out = P[0];
                E.fmt = fmt;
                E.layout_col = 1;
                cur = 0;
            }
            return QSIM_OK;
        }
        E.out = S;
        E.fmt = split ? fmt : FMT_F32;
        E.layout_col = split ? 0 : 1;
        Gj.n = n;
        Gj.cfg = cfg;
        Gj.tiles = tiles_of(n, cfg);
        if (Gj.tiles < 1) return fail(QSIM_E_INVALID, "tile edge %d does not fit n = %d", cfg, n);
        Gj.tile_begin = 0;
        if (!split) {
            Gj.X = S;
            Gj.Y = X[(k - j) & 1];
            Gj.D0 = X[(k - 1 - j) & 1];
            Gj.D1 = nullptr;
        } else if (j < k - 1) {
            Gj.X = P[cur];
            Gj.Y = S;
            Gj.D0 = P[cur ^ 1];
            Gj.D1 = nullptr;
            cur ^= 1;
        } else {
            Gj.X = S;
            Gj.Y = P[cur];
            Gj.D0 = nullptr;
            Gj.D1 = U;
        }
        has_gemm = true;
        return QSIM_OK;
    }
};

}  // namespace qsim
