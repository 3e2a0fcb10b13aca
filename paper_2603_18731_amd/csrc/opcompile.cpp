// Host-side operator compiler: fermionic normal ordering and merging, extended
// Jordan-Wigner transform, combination of equal words, grouping by off-diagonal structure
// and ladder-integer sorting (Methods, Hamiltonian representations; Supplemental Table S1).
// Also builds the host images of the device group / term tables.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>

#include "common.h"

namespace qsd {

bool exact_tags_ok(const std::vector<uint64_t> &z, int W, int64_t N, int64_t C) {
    const int n_qubits = (int)z.size();
    if (W != 1 || N >= (1ll << 26) || n_qubits > 64) return false;
    const uint64_t P = (uint64_t)(C - 1) | 0xFFFFFFFF00000000ull;  // home-slot bits and tag bits
    uint64_t piv[64] = {0};  // piv[b]: the basis vector whose leading bit is b
    for (int q = 0; q < n_qubits; ++q) {
        uint64_t v = z[q] & P;
        int b = 63;
        while (v) {
            while (!((v >> b) & 1ull)) --b;  // leading bit of v
            if (!piv[b]) {
                piv[b] = v;
                break;
            }
            v ^= piv[b];  // clears bit b and leaves only lower bits
        }
        if (!v) return false;  // reduced to zero: dependent on earlier qubits
    }
    return true;
}

uint64_t qubit_hash_value(int q) {
    // splitmix64 output for counter q (Steele, Lea, Flood 2014): fixed pseudo-random words
    uint64_t z = 0x243F6A8885A308D3ull + (uint64_t)(q + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void hash_words(int n_qubits, std::vector<uint64_t> &z) {
    z.resize(n_qubits);
    for (int q = 0; q < n_qubits; ++q) z[q] = qubit_hash_value(q);
}

void part_words(int n_qubits, int split, std::vector<uint32_t> &pz) {
    pz.assign(n_qubits, 0u);
    if (split <= 0) return;
    const int nlo = split, nhi = n_qubits - split;
    for (int q = 0; q < n_qubits; ++q) {
        const bool lo = q < split;
        const int k = lo ? q : q - split;
        // a part of at most 16 qubits is indexed by its own bits (no false passes); a longer
        // one by a pseudo-random 16-bit linear image (another splitmix64 stream)
        const uint32_t v = (lo ? nlo : nhi) <= 16 ? (1u << k) : (uint32_t)(qubit_hash_value(q + 65536) & 0xFFFFu);
        pz[q] = lo ? v : (v << 16);
    }
}

void hash_byte_tables(int Wp, const std::vector<uint64_t> &z, std::vector<uint64_t> &tab) {
    tab.assign((size_t)Wp * 8 * 256, 0);
    for (int c = 0; c < Wp * 8; ++c)
        for (int v = 0; v < 256; ++v) {
            uint64_t h = 0;
            for (int b = 0; b < 8; ++b)
                if ((v >> b & 1) && 8 * c + b < (int)z.size()) h ^= z[8 * c + b];
            tab[(size_t)c * 256 + v] = h;
        }
}

std::vector<uint32_t> group_parts(const qsd_op *op, const std::vector<uint32_t> &pz) {
    const int Wp = op->Wp;
    const size_t G = op->g_mask.size() / (size_t)Wp;
    std::vector<uint32_t> out(G, 0u);
    for (size_t g = 0; g < G; ++g)
        for (int w = 0; w < Wp; ++w)
            for (uint64_t m = op->g_mask[g * Wp + w]; m; m &= m - 1)
                out[g] ^= pz[64 * w + __builtin_ctzll(m)];
    return out;
}

std::vector<uint64_t> group_hashes(const qsd_op *op, const std::vector<uint64_t> &z) {
    const int Wp = op->Wp;
    const size_t G = op->g_mask.size() / (size_t)Wp;
    std::vector<uint64_t> out(G, 0);
    for (size_t g = 0; g < G; ++g)
        for (int w = 0; w < Wp; ++w)
            for (uint64_t m = op->g_mask[g * Wp + w]; m; m &= m - 1)
                out[g] ^= z[64 * w + __builtin_ctzll(m)];
    return out;
}

}  // namespace qsd

using namespace qsd;

namespace {

using cplx = std::complex<double>;

// Merge of two single-mode letters in product order (left, right) over {-, +, 0, 1}, codes
// 5, 6, 1, 2.  Returns the merged letter or -1 when the product vanishes (Table S1).
int merge_letters(int left, int right) {
    auto id = [](int c) { return c == QSD_LOWER ? 0 : c == QSD_RAISE ? 1 : c == QSD_P0 ? 2 : 3; };
    // rows: left in {-, +, 0, 1}; columns: right in {-, +, 0, 1}
    static const int table[4][4] = {
        /* -  */ {-1, QSD_P0, -1, QSD_LOWER},
        /* +  */ {QSD_P1, -1, QSD_RAISE, -1},
        /* 0  */ {QSD_LOWER, -1, QSD_P0, -1},
        /* 1  */ {-1, QSD_RAISE, -1, QSD_P1},
    };
    return table[id(left)][id(right)];
}

// Fermionic product (mode, f/f^dagger) in product order -> qubit word and sign.
// Returns false when the product is identically zero.
bool fermion_to_word(std::vector<Letter> ops, std::vector<Letter> &word, double &sign) {
    sign = 1.0;
    // stable insertion sort by mode; every exchange of two operators on different modes
    // contributes a factor -1
    for (size_t i = 1; i < ops.size(); ++i) {
        for (size_t j = i; j > 0 && ops[j - 1].q > ops[j].q; --j) {
            std::swap(ops[j - 1], ops[j]);
            sign = -sign;
        }
    }
    // merge runs on one mode
    std::vector<Letter> merged;
    for (size_t i = 0; i < ops.size();) {
        size_t j = i;
        int cur = ops[i].code;
        for (j = i + 1; j < ops.size() && ops[j].q == ops[i].q; ++j) {
            cur = merge_letters(cur, ops[j].code);
            if (cur < 0) return false;
        }
        merged.push_back({ops[i].q, (uint8_t)cur});
        i = j;
    }
    // Jordan-Wigner: every ladder letter on mode m carries Z on all qubits below m.  On a
    // qubit of the term the letter stands left of the Z factors of higher ladders, so '-' and
    // '1' (column bit 1) pick up (-1)^{#ladders above}; other qubits get Z when that count is odd.
    word.clear();
    int above = 0;
    std::vector<Letter> rev;
    for (size_t a = merged.size(); a-- > 0;) {
        const Letter &L = merged[a];
        int hi = (a + 1 < merged.size()) ? merged[a + 1].q : -1;
        // qubits strictly between this letter and the next higher letter
        if (hi >= 0 && (above & 1))
            for (int q = hi - 1; q > L.q; --q) rev.push_back({q, QSD_Z});
        if ((L.code == QSD_LOWER || L.code == QSD_P1) && (above & 1)) sign = -sign;
        rev.push_back(L);
        if (L.code == QSD_LOWER || L.code == QSD_RAISE) ++above;
    }
    if (!merged.empty() && (above & 1))
        for (int q = merged.front().q - 1; q >= 0; --q) rev.push_back({q, QSD_Z});
    word.assign(rev.rbegin(), rev.rend());
    return true;
}

bool word_less(const std::vector<Letter> &a, const std::vector<Letter> &b) {
    if (a.size() != b.size()) return a.size() < b.size();
    for (size_t i = 0; i < a.size(); ++i) {
        if (a[i].q != b[i].q) return a[i].q < b[i].q;
        if (a[i].code != b[i].code) return a[i].code < b[i].code;
    }
    return false;
}
bool word_eq(const std::vector<Letter> &a, const std::vector<Letter> &b) {
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i)
        if (a[i].q != b[i].q || a[i].code != b[i].code) return false;
    return true;
}

std::string word_key(const std::vector<Letter> &w) {
    std::string s;
    s.reserve(w.size() * 5);
    for (auto &l : w) {
        char buf[5];
        std::memcpy(buf, &l.q, 4);
        buf[4] = (char)l.code;
        s.append(buf, 5);
    }
    return s;
}

struct Masks {
    std::vector<uint64_t> off, care, want, sgn;
    int ny = 0;
};

Masks masks_of(const std::vector<Letter> &w, int Wp) {
    Masks m;
    m.off.assign(Wp, 0);
    m.care.assign(Wp, 0);
    m.want.assign(Wp, 0);
    m.sgn.assign(Wp, 0);
    for (auto &l : w) {
        uint64_t bit = 1ull << (l.q & 63);
        int k = l.q >> 6;
        switch (l.code) {
            case QSD_Z: m.sgn[k] |= bit; break;
            case QSD_P0: m.care[k] |= bit; break;
            case QSD_P1: m.care[k] |= bit; m.want[k] |= bit; break;
            case QSD_X: m.off[k] |= bit; break;
            case QSD_Y: m.off[k] |= bit; m.sgn[k] |= bit; m.ny++; break;
            case QSD_LOWER: m.off[k] |= bit; m.care[k] |= bit; break;             // row bit 0
            case QSD_RAISE: m.off[k] |= bit; m.care[k] |= bit; m.want[k] |= bit; break;  // row bit 1
        }
    }
    return m;
}

// c' = c * (-i)^{#Y}: with <r|Y|1-r> = -i (-1)^r the Y letters contribute this constant and
// a sign from the row bit, which the sign mask carries.
cplx eff_coef(cplx c, int ny) {
    static const cplx pw[4] = {cplx(1, 0), cplx(0, -1), cplx(-1, 0), cplx(0, 1)};
    return c * pw[ny & 3];
}

int popcount_words(const std::vector<uint64_t> &m) {
    int c = 0;
    for (auto w : m) c += __builtin_popcountll(w);
    return c;
}

bool mask_less(const std::vector<uint64_t> &a, const std::vector<uint64_t> &b) {
    for (size_t w = a.size(); w-- > 0;)
        if (a[w] != b[w]) return a[w] < b[w];
    return false;
}

}  // namespace

extern "C" int qsd_op_compile(int32_t n_qubits, int64_t n_terms, const int64_t *term_ptr, const int32_t *op_idx,
                              const uint8_t *op_code, const double *coef_reim, uint32_t flags, double trim_tol,
                              qsd_op **out) {
    clear_error();
    if (!out) return fail(QSD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_qubits < 1) return fail(QSD_ERR_INVALID_ARG, "n_qubits must be >= 1");
    if (n_qubits > kMaxWords * 64) return fail(QSD_ERR_UNSUPPORTED, "n_qubits > %d", kMaxWords * 64);
    if (n_terms < 0 || (n_terms > 0 && (!term_ptr || !coef_reim)))
        return fail(QSD_ERR_INVALID_ARG, "bad term arrays");
    if (!(trim_tol >= 0.0)) return fail(QSD_ERR_INVALID_ARG, "trim_tol must be >= 0");
    const bool fermionic = flags & QSD_OP_FERMIONIC;
    const int Wp = padded_words(n_qubits);
    if (n_terms > 0 && term_ptr[0] != 0) return fail(QSD_ERR_INVALID_ARG, "term_ptr[0] must be 0");

    // 0. group trimming (Results, CH4-dimer runs): a group is the set of input terms with the
    //    same flip mask (X, Y and ladder letters of a qubit word; every ladder operator of a
    //    fermionic word flips its mode).  Its matrix elements are bounded by the sum of |c|
    //    over its input terms; groups whose bound is below trim_tol are dropped.
    std::vector<char> keep_term((size_t)std::max<int64_t>(n_terms, 0), 1);
    if (trim_tol > 0.0) {
        std::map<std::vector<uint64_t>, double> bound;
        std::vector<std::vector<uint64_t>> tmask((size_t)n_terms);
        for (int64_t t = 0; t < n_terms; ++t) {
            std::vector<uint64_t> m((size_t)Wp, 0ull);
            for (int64_t k = term_ptr[t]; k < term_ptr[t + 1]; ++k) {
                const int q = op_idx[k], code = op_code[k];
                if (q < 0 || q >= n_qubits) continue;  // rejected below
                const uint64_t bit = 1ull << (q & 63);
                if (fermionic)
                    m[(size_t)(q >> 6)] ^= bit;
                else if (code == QSD_X || code == QSD_Y || code == QSD_LOWER || code == QSD_RAISE)
                    m[(size_t)(q >> 6)] |= bit;
            }
            const double a = std::abs(cplx(coef_reim[2 * t], coef_reim[2 * t + 1]));
            bool any = false;
            for (uint64_t w : m) any |= w != 0;
            if (any) bound[m] += a;
            tmask[(size_t)t] = std::move(m);
        }
        for (int64_t t = 0; t < n_terms; ++t) {
            auto it = bound.find(tmask[(size_t)t]);
            if (it != bound.end() && it->second < trim_tol) keep_term[(size_t)t] = 0;
        }
    }

    // 1. per-term normalization --------------------------------------------------------
    std::vector<CompiledTerm> raw;
    raw.reserve((size_t)n_terms);
    std::vector<Letter> ops, word;
    for (int64_t t = 0; t < n_terms; ++t) {
        int64_t a = term_ptr[t], b = term_ptr[t + 1];
        if (b < a) return fail(QSD_ERR_INVALID_ARG, "term_ptr not ascending at term %lld", (long long)t);
        if (b > a && (!op_idx || !op_code)) return fail(QSD_ERR_INVALID_ARG, "op arrays are NULL");
        cplx c(coef_reim[2 * t], coef_reim[2 * t + 1]);
        if (!std::isfinite(c.real()) || !std::isfinite(c.imag()))
            return fail(QSD_ERR_INVALID_ARG, "non-finite coefficient at term %lld", (long long)t);
        ops.clear();
        for (int64_t k = a; k < b; ++k) {
            int q = op_idx[k], code = op_code[k];
            if (q < 0 || q >= n_qubits)
                return fail(QSD_ERR_INVALID_ARG, "term %lld: qubit index %d out of range", (long long)t, q);
            if (fermionic ? (code != QSD_LOWER && code != QSD_RAISE) : (code > QSD_RAISE))
                return fail(QSD_ERR_INVALID_ARG, "term %lld: invalid letter code %d", (long long)t, code);
            ops.push_back({q, (uint8_t)code});
        }
        if (c == cplx(0, 0) || !keep_term[(size_t)t]) continue;
        double sign = 1.0;
        if (fermionic) {
            if (!fermion_to_word(ops, word, sign)) continue;
        } else {
            word = ops;
            std::stable_sort(word.begin(), word.end(), [](const Letter &x, const Letter &y) { return x.q < y.q; });
            for (size_t i = 1; i < word.size(); ++i)
                if (word[i].q == word[i - 1].q)
                    return fail(QSD_ERR_INVALID_ARG, "term %lld: qubit %d repeated in a qubit word", (long long)t,
                                word[i].q);
        }
        raw.push_back({word, c * sign});
    }

    // 2. combine equal words (sort by weight, then word; sums in input order) -------------
    std::vector<size_t> order(raw.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return word_less(raw[x].word, raw[y].word); });
    std::vector<CompiledTerm> comb;
    for (size_t i = 0; i < order.size();) {
        size_t j = i;
        CompiledTerm ct = raw[order[i]];
        for (j = i + 1; j < order.size() && word_eq(raw[order[j]].word, ct.word); ++j) ct.c += raw[order[j]].c;
        comb.push_back(std::move(ct));
        i = j;
    }

    // 3. Hermiticity check ------------------------------------------------------------------
    if (flags & QSD_OP_CHECK_HERMITIAN) {
        std::map<std::string, cplx> coef_of;
        double cmax = 0;
        for (auto &ct : comb) {
            coef_of[word_key(ct.word)] = ct.c;
            cmax = std::max(cmax, std::abs(ct.c));
        }
        for (auto &ct : comb) {
            std::vector<Letter> adj = ct.word;
            for (auto &l : adj)
                if (l.code == QSD_LOWER)
                    l.code = QSD_RAISE;
                else if (l.code == QSD_RAISE)
                    l.code = QSD_LOWER;
            auto it = coef_of.find(word_key(adj));
            cplx ca = it == coef_of.end() ? cplx(0, 0) : it->second;
            if (std::abs(ca - std::conj(ct.c)) > 1e-12 * std::max(1.0, cmax))
                return fail(QSD_ERR_NOT_HERMITIAN, "operator is not Hermitian (a word's adjoint has coefficient "
                                                   "(%g,%g), expected (%g,%g))",
                            ca.real(), ca.imag(), ct.c.real(), -ct.c.imag());
        }
    }

    // 4. split diagonal / group off-diagonal by (weight, structure) ---------------------------
    struct Item {
        size_t idx;
        Masks m;
        int weight;
        int part_class = 0;                 // by parts: 0 low half only, 1 both, 2 high half only
        std::vector<uint64_t> lo, hi;       // by parts: the flip mask's halves
    };
    std::vector<Item> diag, offd;
    for (size_t i = 0; i < comb.size(); ++i) {
        Masks m = masks_of(comb[i].word, Wp);
        int wgt = popcount_words(m.off);
        if (wgt == 0)
            diag.push_back({i, std::move(m), 0});
        else
            offd.push_back({i, std::move(m), wgt});
    }
    const bool by_mask = (flags & QSD_OP_ORDER_BY_MASK) != 0;
    const bool by_parts = (flags & QSD_OP_ORDER_BY_PARTS) != 0;
    if (by_parts) {
        // the flip mask split at qubit n/2 into its low and high halves; groups ordered by which
        // halves they flip (low only, both, high only); groups flipping both by the high half,
        // then weight, then the low half (runs that flip the high part alike); the others by
        // weight, then mask (short and long term ranges apart)
        const int half = n_qubits / 2;
        for (auto &it : offd) {
            it.lo.assign(it.m.off.size(), 0);
            it.hi.assign(it.m.off.size(), 0);
            for (size_t w = 0; w < it.m.off.size(); ++w)
                for (uint64_t b = it.m.off[w]; b; b &= b - 1) {
                    const int q = 64 * (int)w + __builtin_ctzll(b);
                    (q < half ? it.lo : it.hi)[w] |= 1ull << (q & 63);
                }
            const bool l = popcount_words(it.lo) > 0, h = popcount_words(it.hi) > 0;
            it.part_class = l && h ? 1 : (h ? 2 : 0);
        }
    }
    std::stable_sort(offd.begin(), offd.end(), [&](const Item &x, const Item &y) {
        if (by_parts) {
            if (x.part_class != y.part_class) return x.part_class < y.part_class;
            if (x.part_class == 1 && x.hi != y.hi) return mask_less(x.hi, y.hi);
            if (x.weight != y.weight) return x.weight < y.weight;
            if (x.hi != y.hi) return mask_less(x.hi, y.hi);
            return mask_less(x.lo, y.lo);
        }
        if (!by_mask && x.weight != y.weight) return x.weight < y.weight;
        return mask_less(x.m.off, y.m.off);
    });

    auto *op = new (std::nothrow) qsd_op();
    if (!op) return fail(QSD_ERR_OUT_OF_MEMORY, "host allocation failed");
    op->n_qubits = n_qubits;
    op->Wp = Wp;
    bool cplx_mat = (flags & QSD_OP_FORCE_COMPLEX) != 0;

    auto push_cws = [&](std::vector<uint64_t> &dst, const Masks &m) {
        dst.insert(dst.end(), m.care.begin(), m.care.end());
        dst.insert(dst.end(), m.want.begin(), m.want.end());
        dst.insert(dst.end(), m.sgn.begin(), m.sgn.end());
    };
    auto push_coef = [&](std::vector<double> &dst, cplx c, int ny) {
        cplx e = eff_coef(c, ny);
        if (e.imag() != 0.0) cplx_mat = true;
        dst.push_back(e.real());
        dst.push_back(e.imag());
    };

    // diagonal group
    op->group_ptr.push_back(0);
    for (auto &it : diag) {
        op->terms.push_back(comb[it.idx]);
        push_cws(op->diag_cws, it.m);
        push_coef(op->diag_coef, comb[it.idx].c, it.m.ny);
    }
    op->group_ptr.push_back((int64_t)op->terms.size());
    op->group_ladder.push_back(0);

    const bool no_ladder = flags & QSD_OP_NO_LADDER_INT;
    for (size_t i = 0; i < offd.size();) {
        size_t j = i + 1;
        while (j < offd.size() && offd[j].m.off == offd[i].m.off) ++j;
        // group [i, j)
        const std::vector<uint64_t> &M = offd[i].m.off;
        std::vector<int> pos;
        for (int w = 0; w < Wp; ++w)
            for (int b = 0; b < 64; ++b)
                if (M[w] >> b & 1) pos.push_back(64 * w + b);
        bool ladder = !no_ladder && (int)pos.size() <= kMaxLadder && (j - i) <= 65535;
        std::vector<int> lint(j - i, 0);
        for (size_t a = i; a < j && ladder; ++a) {
            const auto &w = comb[offd[a].idx].word;
            int L = 0;
            for (size_t k = 0; k < pos.size(); ++k) {
                auto itl = std::find_if(w.begin(), w.end(), [&](const Letter &l) { return l.q == pos[k]; });
                if (itl->code == QSD_RAISE)
                    L |= 1 << k;
                else if (itl->code != QSD_LOWER)
                    ladder = false;
            }
            lint[a - i] = L;
        }
        std::vector<size_t> ord(j - i);
        std::iota(ord.begin(), ord.end(), 0);
        if (ladder) std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return lint[x] < lint[y]; });
        // Strings of at most 32 qubits: inside each ladder range, the terms whose only care bit
        // beyond the flip mask is one qubit r that they want set (a spectator's number operator
        // after the Jordan-Wigner transform) move behind the others, one per qubit, by r; the
        // range's first term records those qubits.  A row then visits only the tail terms of the
        // qubits it has set (the others cannot match), and every row's sum still adds the terms
        // that match in the order they are stored.
        std::vector<uint32_t> tail_at(j - i, 0u);  // by position in ord
        if (ladder && Wp == 1 && n_qubits <= 32) {
            auto spectator = [&](size_t a) -> int {  // r, or -1
                const Masks &m = offd[i + a].m;
                const uint64_t extra = m.care[0] & ~M[0];
                if (!extra || (extra & (extra - 1)) || !(m.want[0] & extra)) return -1;
                return __builtin_ctzll(extra);
            };
            for (size_t a = 0; a < ord.size();) {
                size_t b = a;
                while (b < ord.size() && lint[ord[b]] == lint[ord[a]]) ++b;
                std::vector<size_t> plain, tail;
                uint32_t R = 0;
                for (size_t u = a; u < b; ++u) {
                    const int r = spectator(ord[u]);
                    if (r >= 0 && r < 32 && !((R >> r) & 1u)) {
                        tail.push_back(ord[u]);
                        R |= 1u << r;
                    } else {
                        plain.push_back(ord[u]);
                    }
                }
                std::stable_sort(tail.begin(), tail.end(),
                                 [&](size_t x, size_t y) { return spectator(x) < spectator(y); });
                std::copy(plain.begin(), plain.end(), ord.begin() + a);
                std::copy(tail.begin(), tail.end(), ord.begin() + a + plain.size());
                tail_at[a] = R;
                a = b;
            }
        }

        uint32_t term0 = (uint32_t)(op->t_coef.size() / 2);
        bool care = false;
        for (size_t r = 0; r < ord.size(); ++r) {
            const Item &it = offd[i + ord[r]];
            op->t_tail.push_back(tail_at[r]);
            op->terms.push_back(comb[it.idx]);
            push_cws(op->t_cws, it.m);
            push_coef(op->t_coef, comb[it.idx].c, it.m.ny);
            for (int w = 0; w < Wp; ++w) {
                uint64_t extra = it.m.care[w] & (ladder ? ~M[w] : ~0ull);
                if (extra) care = true;
            }
        }
        uint16_t iptr[kIptr] = {0};
        uint32_t live = 0;
        if (ladder) {
            for (int L = 0; L <= 16; ++L) {
                size_t cnt = 0;
                for (size_t r = 0; r < ord.size(); ++r)
                    if (lint[ord[r]] < L) ++cnt;
                iptr[L] = (uint16_t)cnt;
            }
            for (int L = 0; L < 16; ++L)
                if (iptr[L + 1] > iptr[L]) live |= 1u << L;
        }
        uint64_t gpos = 0;
        for (size_t k = 0; k < pos.size() && k < 4; ++k) gpos |= (uint64_t)pos[k] << (16 * k);
        op->g_mask.insert(op->g_mask.end(), M.begin(), M.end());
        op->g_pos.push_back(gpos);
        // Scan record.  The device forms a 4-bit ladder integer from four positions (unused
        // ones repeat qubit j's bit, so they are don't-cares): bits 0..15 hold the live table
        // replicated over the don't-care bits (all ones for groups scanned term by term);
        // bits 16 + 12j hold p_j - j, the right shift that brings qubit p_j to bit j.
        {
            uint64_t rec = 0;
            const int kk = ladder ? (int)pos.size() : 0;
            for (int L = 0; L < 16; ++L) {
                const int Lk = kk ? (L & ((1 << kk) - 1)) : 0;
                const bool lv = ladder ? ((live >> Lk) & 1u) : true;
                if (lv) rec |= 1ull << L;
            }
            for (int j = 0; j < 4; ++j) {
                const int p = (ladder && j < kk) ? pos[j] : j;
                rec |= (uint64_t)(p - j) << (16 + 12 * j);
            }
            op->g_scan.push_back(rec);
        }
        op->g_info.push_back((uint32_t)(ladder ? pos.size() : 0) | (ladder ? kInfoLadder : 0) |
                             (care ? kInfoCare : 0) | (live << 16));
        op->g_term0.push_back(term0);
        op->g_nterm.push_back((uint32_t)(j - i));
        op->g_iptr.insert(op->g_iptr.end(), iptr, iptr + kIptr);
        op->group_ptr.push_back((int64_t)op->terms.size());
        op->group_ladder.push_back(ladder ? 1 : 0);
        op->max_group_terms = std::max<int64_t>(op->max_group_terms, (int64_t)(j - i));
        i = j;
    }
    // the device reads scan records 8 at a time
    while (op->g_scan.size() % 8 != 0 || op->g_scan.size() < op->g_info.size() + 8) op->g_scan.push_back(0);
    op->is_complex = cplx_mat;
    *out = op;
    return QSD_OK;
}

extern "C" int qsd_op_info(const qsd_op *op, int64_t *T, int64_t *n_letters, int64_t *G, int32_t *is_complex,
                           int32_t *n_qubits) {
    clear_error();
    if (!op) return fail(QSD_ERR_INVALID_ARG, "op is NULL");
    if (T) *T = (int64_t)op->terms.size();
    if (n_letters) {
        int64_t n = 0;
        for (auto &t : op->terms) n += (int64_t)t.word.size();
        *n_letters = n;
    }
    if (G) *G = (int64_t)op->group_ladder.size();
    if (is_complex) *is_complex = op->is_complex ? 1 : 0;
    if (n_qubits) *n_qubits = op->n_qubits;
    return QSD_OK;
}

extern "C" int qsd_op_export(const qsd_op *op, int64_t *term_ptr, int32_t *op_idx, uint8_t *op_code,
                             double *coef_reim, int64_t *group_ptr, int32_t *group_ladder) {
    clear_error();
    if (!op) return fail(QSD_ERR_INVALID_ARG, "op is NULL");
    int64_t k = 0;
    if (term_ptr) term_ptr[0] = 0;
    for (size_t t = 0; t < op->terms.size(); ++t) {
        for (auto &l : op->terms[t].word) {
            if (op_idx) op_idx[k] = l.q;
            if (op_code) op_code[k] = l.code;
            ++k;
        }
        if (term_ptr) term_ptr[t + 1] = k;
        if (coef_reim) {
            coef_reim[2 * t] = op->terms[t].c.real();
            coef_reim[2 * t + 1] = op->terms[t].c.imag();
        }
    }
    if (group_ptr) std::copy(op->group_ptr.begin(), op->group_ptr.end(), group_ptr);
    if (group_ladder) std::copy(op->group_ladder.begin(), op->group_ladder.end(), group_ladder);
    return QSD_OK;
}

extern "C" int qsd_op_destroy(qsd_op *op) {
    clear_error();
    delete op;
    return QSD_OK;
}
