// Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the library's host core
// (operator compiler, hash and part-filter word generators, error state).  Built by the host
// tests with g++ only; it makes no HIP call.
//
// It compiles random qubit and fermionic operators of 1 to 1024 qubits through qsd_op_compile,
// reads them back with qsd_op_info / qsd_op_export, derives the hash and part-filter tables the
// device tables are built from, and drives every argument check of the compiler.  Any
// out-of-bounds access, use after free, leak or undefined operation aborts with the sanitizer's
// report; the last line printed on success is "host core clean".
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "common.h"

namespace {

int g_failures = 0;

void expect(bool ok, const char *what) {
    if (!ok) {
        std::printf("FAILED: %s (%s)\n", what, qsd_last_error());
        ++g_failures;
    }
}

struct Terms {
    std::vector<int64_t> ptr{0};
    std::vector<int32_t> idx;
    std::vector<uint8_t> code;
    std::vector<double> coef;
    int64_t n() const { return (int64_t)ptr.size() - 1; }
};

// Random Hermitian operator: every word comes with its adjoint and the conjugate coefficient.
Terms random_ops(std::mt19937_64 &rng, int n, int nterms, bool fermionic) {
    Terms t;
    std::uniform_int_distribution<int> q(0, n - 1), len(0, 4), letter(0, 6), fl(5, 6);
    std::normal_distribution<double> c(0.0, 1.0);
    for (int k = 0; k < nterms; ++k) {
        const int m = len(rng);
        std::vector<int32_t> qs;
        std::vector<uint8_t> cs;
        for (int j = 0; j < m; ++j) {
            int qq = q(rng);
            if (!fermionic) {  // distinct qubits in qubit mode
                bool dup = false;
                for (int32_t x : qs) dup |= x == qq;
                if (dup) continue;
            }
            qs.push_back(qq);
            cs.push_back((uint8_t)(fermionic ? fl(rng) : letter(rng)));
        }
        const double re = c(rng), im = fermionic ? 0.0 : c(rng);
        for (int pass = 0; pass < 2; ++pass) {
            for (size_t j = 0; j < qs.size(); ++j) {
                // adjoint: reversed product order for fermions, 5 <-> 6 swapped, Y -> Y
                const size_t jj = (pass && fermionic) ? qs.size() - 1 - j : j;
                uint8_t cc = cs[jj];
                if (pass && (cc == 5 || cc == 6)) cc = (uint8_t)(11 - cc);
                t.idx.push_back(qs[jj]);
                t.code.push_back(cc);
            }
            t.ptr.push_back((int64_t)t.idx.size());
            t.coef.push_back(re);
            t.coef.push_back(pass ? -im : im);
        }
    }
    return t;
}

void compile_and_read(const Terms &t, int n, uint32_t flags) {
    qsd_op *op = nullptr;
    const int rc = qsd_op_compile(n, t.n(), t.ptr.data(), t.idx.data(), t.code.data(), t.coef.data(), flags, 0.0, &op);
    expect(rc == QSD_OK, "compile");
    if (rc != QSD_OK) return;
    int64_t T = 0, L = 0, G = 0;
    int32_t cplx = 0, nq = 0;
    expect(qsd_op_info(op, &T, &L, &G, &cplx, &nq) == QSD_OK, "info");
    expect(nq == n, "n_qubits round trip");
    std::vector<int64_t> tp(T + 1), gp(G + 1);
    std::vector<int32_t> oi(L), gl(G);
    std::vector<uint8_t> oc(L);
    std::vector<double> cf(2 * T);
    expect(qsd_op_export(op, tp.data(), oi.data(), oc.data(), cf.data(), gp.data(), gl.data()) == QSD_OK, "export");
    expect(tp[T] == L && gp[G] == T, "export sizes");
    for (int64_t l = 0; l < L; ++l) expect(oi[l] >= 0 && oi[l] < n && oc[l] <= 6, "exported letter in range");
    // the tables the device path is built from
    std::vector<uint64_t> z, tab;
    qsd::hash_words(n, z);
    expect((int)z.size() == n, "hash words");
    const int Wp = qsd::padded_words(n);
    qsd::hash_byte_tables(Wp, z, tab);
    (void)qsd::group_hashes(op, z);
    for (int split : {1, n / 2, n - 1}) {
        if (split < 1 || split >= n) continue;
        std::vector<uint32_t> pz;
        qsd::part_words(n, split, pz);
        (void)qsd::group_parts(op, pz);
    }
    (void)qsd::exact_tags_ok(z, (n + 63) / 64, 1000, 1 << 16);
    expect(qsd_op_destroy(op) == QSD_OK, "destroy");
}

void argument_checks() {
    const int64_t ptr[2] = {0, 1};
    const int32_t idx[1] = {0};
    const uint8_t code[1] = {3};
    const uint8_t bad_code[1] = {9};
    const int32_t bad_idx[1] = {12};
    const double coef[2] = {1.0, 0.0};
    qsd_op *op = nullptr;
    expect(qsd_op_compile(0, 1, ptr, idx, code, coef, 0, 0.0, &op) != QSD_OK, "n_qubits 0 rejected");
    expect(qsd_op_compile(qsd_max_qubits() + 1, 1, ptr, idx, code, coef, 0, 0.0, &op) != QSD_OK, "too many qubits");
    expect(qsd_op_compile(4, -1, ptr, idx, code, coef, 0, 0.0, &op) != QSD_OK, "negative term count");
    expect(qsd_op_compile(4, 1, nullptr, idx, code, coef, 0, 0.0, &op) != QSD_OK, "NULL term_ptr");
    expect(qsd_op_compile(4, 1, ptr, idx, bad_code, coef, 0, 0.0, &op) != QSD_OK, "letter code out of range");
    expect(qsd_op_compile(4, 1, ptr, bad_idx, code, coef, 0, 0.0, &op) != QSD_OK, "qubit out of range");
    expect(qsd_op_compile(4, 1, ptr, idx, code, coef, QSD_OP_FERMIONIC, 0.0, &op) != QSD_OK, "X in fermionic mode");
    expect(qsd_op_compile(4, 1, ptr, idx, code, coef, 0, 0.0, nullptr) != QSD_OK, "NULL output");
    expect(std::strlen(qsd_last_error()) > 0, "error message set");
    // a non-Hermitian word under the Hermiticity check
    const uint8_t raise[1] = {6};
    expect(qsd_op_compile(4, 1, ptr, idx, raise, coef, QSD_OP_CHECK_HERMITIAN, 0.0, &op) == QSD_ERR_NOT_HERMITIAN,
           "Hermiticity check");
    expect(qsd_op_info(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) != QSD_OK, "info of NULL");
    (void)qsd_op_destroy(nullptr);  // must not crash
}

}  // namespace

int main() {
    std::mt19937_64 rng(20260318);
    argument_checks();
    for (int n : {1, 2, 5, 16, 32, 63, 64, 65, 130, 200, 513, 1024}) {
        for (int rep = 0; rep < 3; ++rep) {
            const Terms q = random_ops(rng, n, 40, false);
            compile_and_read(q, n, QSD_OP_CHECK_HERMITIAN);
            compile_and_read(q, n, QSD_OP_ORDER_BY_MASK | QSD_OP_FORCE_COMPLEX);
            compile_and_read(q, n, QSD_OP_NO_LADDER_INT);
            const Terms f = random_ops(rng, n, 40, true);
            compile_and_read(f, n, QSD_OP_FERMIONIC | QSD_OP_CHECK_HERMITIAN);
            compile_and_read(f, n, QSD_OP_FERMIONIC | QSD_OP_ORDER_BY_MASK);
        }
    }
    // an empty operator and a zero-coefficient-only one
    Terms e;
    compile_and_read(e, 8, 0);
    Terms zc;
    zc.idx = {0, 1};
    zc.code = {3, 3};
    zc.ptr = {0, 2};
    zc.coef = {0.0, 0.0};
    compile_and_read(zc, 8, 0);
    if (g_failures) {
        std::printf("%d checks failed\n", g_failures);
        return 1;
    }
    std::printf("host core clean\n");
    return 0;
}
