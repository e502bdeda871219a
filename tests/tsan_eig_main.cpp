// Drives the host eigensolver of a libpkm whose host code carries
// ThreadSanitizer (built with --host-tsan) from a program built with
// -fsanitize=thread: symmetric matrices around the 64-column blocks of the
// threaded rotation pass, each checked by its reconstruction.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "pkm.h"

int main() {
    for (int n : {65, 130, 300}) {
        std::mt19937_64 gen(n);
        std::normal_distribution<double> nd;
        std::vector<double> A(size_t(n) * n), w(n), Z(size_t(n) * n);
        double amax = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j <= i; ++j) {
                A[size_t(i) * n + j] = A[size_t(j) * n + i] = nd(gen);
                amax = std::fmax(amax, std::fabs(A[size_t(i) * n + j]));
            }
        if (pkm_sym_eig(n, A.data(), w.data(), Z.data()) != PKM_OK) return 2;
        double err = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int c = 0; c < n; ++c) s += Z[size_t(i) * n + c] * w[c] * Z[size_t(j) * n + c];
                err = std::fmax(err, std::fabs(s - A[size_t(i) * n + j]));
            }
        if (!(err < 1e-10 * amax)) {
            std::printf("n = %d: reconstruction error %g\n", n, err);
            return 3;
        }
    }
    std::puts("tsan run clean");
    return 0;
}
