// libnf_serial.so: the serial CPU algorithms of Section 3 (include/nf_serial.h).
//
// The table D(i, j), 1 <= i <= j <= n, of Eq. 1 is kept twice, row-major and
// transposed, so that the row cells D(i, k-1) and the column cells D(k, j) of
// a cell's split points are both read contiguously.  Entries with j < i are
// the boundary zeros D(i, i-1) = 0.
//
// Difference vectors (Lemma 1 keeps them 0/1):
//   row group K of row i:    base D(i, Kq), bit p-1 = D(i, Kq+p) - D(i, Kq+p-1)
//   column group K of col j: base D(Kq+1, j), bit p-1 = D(Kq+p, j) - D(Kq+p+1, j)
// for p = 1 .. q-1.  With them the q split points k = Kq+1 .. Kq+q of cell
// (i, j) give (Eq. 3)
//   max_k D(i, k-1) + D(k, j) = rowbase + colbase + R[h][c],
//   R[h][c] = max over t = 0..q-1 of sum_{p<=t} (h_p - c_p).
// A row group is finished with the cell D(i, Kq+q-1), a column group with the
// cell D(Kq+1, j); in both fill orders every cell that looks a group up comes
// after that cell.
#include "nf_serial.h"

#include <omp.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

namespace {

int code_of(char ch)
{
    switch (ch) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'U': case 'u': return 3;
    default: return -1;
    }
}

// Best prefix total of Eq. 3 for one pair of difference vectors (m = q-1 bits).
inline int best_prefix(unsigned h, unsigned c, int m)
{
    int run = 0, best = 0;
    for (int p = 0; p < m; ++p) {
        run += (int)((h >> p) & 1u) - (int)((c >> p) & 1u);
        if (run > best) best = run;
    }
    return best;
}

struct Fold {
    int n = 0, q = 1, m = 0, W = 0, NG = 0, S = 1;
    int variant = 0;
    std::vector<uint8_t> code;    // code[1..n]
    std::vector<int16_t> D, DT;   // D[i*W + j] = D(i, j) = DT[j*W + i]
    std::vector<int16_t> rb, cb;  // row / column group bases [i*NG + K], [j*NG + K]
    std::vector<uint16_t> rh, cc; // row / column group bits
    std::vector<uint8_t> R;       // [h*S + c]; 0xff = not built yet (memoized variants)
    std::vector<uint8_t> row_built;  // partial memo: row h of R built
    std::vector<int16_t> fg;      // FG: [(i*NG + K)*S + c] = rowbase + best prefix
    int64_t lookups = 0, splits = 0, r_entries = 0, vectors = 0;

    int16_t d(int i, int j) const { return D[(size_t)i * W + j]; }
};

// One cell.  Returns D(i, j) and adds its work to the counters passed.
template <int V>
inline int cell(Fold& f, int i, int j, int64_t& lk, int64_t& sp, int64_t& re)
{
    const int16_t* row = &f.D[(size_t)i * f.W];   // row[k-1] = D(i, k-1)
    const int16_t* col = &f.DT[(size_t)j * f.W];  // col[k]   = D(k, j)
    int best = (f.code[i] + f.code[j] == 3 ? 1 : 0) + f.d(i + 1, j - 1);
    auto plain = [&](int k0, int k1) {  // split points k0 .. k1
        int b = best;
        for (int k = k0; k <= k1; ++k) b = std::max(b, (int)row[k - 1] + (int)col[k]);
        best = b;
        sp += k1 >= k0 ? k1 - k0 + 1 : 0;
    };
    if (V == NF_SERIAL_PLAIN) {
        plain(i + 1, j);
        return best;
    }
    const int q = f.q;
    const int Klo = (i + q - 1) / q, Khi = j / q - 1;
    if (Klo > Khi) {
        plain(i + 1, j);
        return best;
    }
    plain(i + 1, Klo * q);
    plain((Khi + 1) * q + 1, j);
    const int16_t* RB = &f.rb[(size_t)i * f.NG];
    const uint16_t* RH = &f.rh[(size_t)i * f.NG];
    const int16_t* CB = &f.cb[(size_t)j * f.NG];
    const uint16_t* CC = &f.cc[(size_t)j * f.NG];
    const int S = f.S;
    int b = best;
    if (V == NF_SERIAL_TWO_VECTOR || V == NF_SERIAL_PARTIAL_MEMO) {
        const uint8_t* R = f.R.data();
        for (int K = Klo; K <= Khi; ++K) b = std::max(b, RB[K] + CB[K] + (int)R[(size_t)RH[K] * S + CC[K]]);
    } else if (V == NF_SERIAL_FULL_MEMO) {
        uint8_t* R = f.R.data();
        for (int K = Klo; K <= Khi; ++K) {
            uint8_t& r = R[(size_t)RH[K] * S + CC[K]];
            if (r == 0xff) {
                r = (uint8_t)best_prefix(RH[K], CC[K], f.m);
                ++re;
            }
            b = std::max(b, RB[K] + CB[K] + (int)r);
        }
    } else {  // NF_SERIAL_FG
        const int16_t* T = &f.fg[(size_t)i * f.NG * S];
        for (int K = Klo; K <= Khi; ++K) b = std::max(b, (int)T[(size_t)K * S + CC[K]] + CB[K]);
    }
    lk += Khi - Klo + 1;
    return b;
}

// Store D(i, j) and the difference vectors it finishes.
template <int V>
inline void finish(Fold& f, int i, int j, int v, int64_t& vec, int64_t& re)
{
    f.D[(size_t)i * f.W + j] = (int16_t)v;
    f.DT[(size_t)j * f.W + i] = (int16_t)v;
    if (V == NF_SERIAL_PLAIN) return;
    const int q = f.q, m = f.m;
    if ((j + 1) % q == 0) {  // row group K = D(i, Kq .. Kq+q-1) is finished
        const int K = (j + 1) / q - 1;
        if (K * q >= i) {
            unsigned h = 0;
            for (int p = 1; p <= m; ++p) h |= (unsigned)(f.d(i, K * q + p) - f.d(i, K * q + p - 1)) << (p - 1);
            const int base = f.d(i, K * q);
            f.rb[(size_t)i * f.NG + K] = (int16_t)base;
            f.rh[(size_t)i * f.NG + K] = (uint16_t)h;
            ++vec;
            if (V == NF_SERIAL_PARTIAL_MEMO && !f.row_built[h]) {
                for (int c = 0; c < f.S; ++c) f.R[(size_t)h * f.S + c] = (uint8_t)best_prefix(h, (unsigned)c, m);
                f.row_built[h] = 1;
                re += f.S;
            }
            if (V == NF_SERIAL_FG) {
                int16_t* T = &f.fg[((size_t)i * f.NG + K) * f.S];
                for (int c = 0; c < f.S; ++c) T[c] = (int16_t)(base + best_prefix(h, (unsigned)c, m));
                re += f.S;
            }
        }
    }
    if (i % q == 1 || q == 1) {  // column group K = D(Kq+1 .. Kq+q, j) is finished
        const int K = (i - 1) / q;
        if (K * q + q <= j) {
            unsigned c = 0;
            for (int p = 1; p <= m; ++p) c |= (unsigned)(f.d(K * q + p, j) - f.d(K * q + p + 1, j)) << (p - 1);
            f.cb[(size_t)j * f.NG + K] = f.d(K * q + 1, j);
            f.cc[(size_t)j * f.NG + K] = (uint16_t)c;
            ++vec;
        }
    }
}

template <int V>
void fill_columns(Fold& f)
{
    int64_t lk = 0, sp = 0, re = 0, vec = 0;
    for (int j = 1; j <= f.n; ++j) {
        finish<V>(f, j, j, 0, vec, re);
        for (int i = j - 1; i >= 1; --i) finish<V>(f, i, j, cell<V>(f, i, j, lk, sp, re), vec, re);
    }
    f.lookups += lk;
    f.splits += sp;
    f.r_entries += re;
    f.vectors += vec;
}

template <int V>
void fill_diagonals(Fold& f, int threads)
{
    int64_t lk = 0, sp = 0, re = 0, vec = 0;
    for (int i = 1; i <= f.n; ++i) finish<V>(f, i, i, 0, vec, re);
    for (int dd = 1; dd < f.n; ++dd) {
#pragma omp parallel for num_threads(threads) schedule(static) reduction(+ : lk, sp, re, vec)
        for (int i = 1; i <= f.n - dd; ++i) {
            const int j = i + dd;
            finish<V>(f, i, j, cell<V>(f, i, j, lk, sp, re), vec, re);
        }
    }
    f.lookups += lk;
    f.splits += sp;
    f.r_entries += re;
    f.vectors += vec;
}

}  // namespace

extern "C" int nf_serial_fold(const char* seq, int n, int q, int variant, int threads, int16_t* S_out,
                              nf_serial_stats_t* stats)
{
    if (n < 0 || n > NF_SERIAL_MAX_N || (n > 0 && !seq) || threads < 1) return NF_SERIAL_E_INVAL;
    if (variant < NF_SERIAL_PLAIN || variant > NF_SERIAL_FG) return NF_SERIAL_E_INVAL;
    if (variant != NF_SERIAL_PLAIN && (q < 1 || q > NF_SERIAL_Q_MAX)) return NF_SERIAL_E_INVAL;
    if (threads > 1 && variant != NF_SERIAL_PLAIN && variant != NF_SERIAL_TWO_VECTOR) return NF_SERIAL_E_INVAL;
    if (variant == NF_SERIAL_PLAIN) q = 1;
    Fold f;
    try {
        f.n = n;
        f.q = q;
        f.m = q - 1;
        f.S = 1 << f.m;
        f.variant = variant;
        f.W = n + 2;
        f.NG = n / q + 2;
        f.code.assign((size_t)n + 2, 0);
        for (int i = 0; i < n; ++i) {
            const int c = code_of(seq[i]);
            if (c < 0) return NF_SERIAL_E_INVAL;
            f.code[i + 1] = (uint8_t)c;
        }
        f.D.assign((size_t)f.W * f.W, 0);
        f.DT.assign((size_t)f.W * f.W, 0);
        if (variant != NF_SERIAL_PLAIN) {
            const size_t groups = (size_t)f.W * f.NG;
            f.rb.assign(groups, 0);
            f.rh.assign(groups, 0);
            f.cb.assign(groups, 0);
            f.cc.assign(groups, 0);
        }
        if (variant == NF_SERIAL_TWO_VECTOR) {  // every pair before the fill
            f.R.resize((size_t)f.S * f.S);
            for (int h = 0; h < f.S; ++h)
                for (int c = 0; c < f.S; ++c) f.R[(size_t)h * f.S + c] = (uint8_t)best_prefix(h, c, f.m);
            f.r_entries = (int64_t)f.S * f.S;
        } else if (variant == NF_SERIAL_PARTIAL_MEMO) {
            f.R.assign((size_t)f.S * f.S, 0);
            f.row_built.assign(f.S, 0);
        } else if (variant == NF_SERIAL_FULL_MEMO) {
            f.R.assign((size_t)f.S * f.S, 0xff);
        } else if (variant == NF_SERIAL_FG) {
            f.fg.assign((size_t)f.W * f.NG * f.S, 0);
        }
    } catch (const std::bad_alloc&) {
        return NF_SERIAL_E_NOMEM;
    }
    switch (variant) {
    case NF_SERIAL_PLAIN:
        if (threads > 1) fill_diagonals<NF_SERIAL_PLAIN>(f, threads); else fill_columns<NF_SERIAL_PLAIN>(f);
        break;
    case NF_SERIAL_TWO_VECTOR:
        if (threads > 1) fill_diagonals<NF_SERIAL_TWO_VECTOR>(f, threads); else fill_columns<NF_SERIAL_TWO_VECTOR>(f);
        break;
    case NF_SERIAL_PARTIAL_MEMO: fill_columns<NF_SERIAL_PARTIAL_MEMO>(f); break;
    case NF_SERIAL_FULL_MEMO: fill_columns<NF_SERIAL_FULL_MEMO>(f); break;
    default: fill_columns<NF_SERIAL_FG>(f); break;
    }
    if (S_out)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) S_out[(size_t)i * n + j] = j >= i ? f.d(i + 1, j + 1) : (int16_t)0;
    if (stats) {
        stats->lookups = f.lookups;
        stats->splits = f.splits;
        stats->r_entries = f.r_entries;
        stats->vectors = f.vectors;
    }
    return n >= 1 ? f.d(1, n) : 0;
}
