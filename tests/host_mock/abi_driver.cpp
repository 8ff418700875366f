// Drives the product entry points on matrices without stored entries
// against the mock HIP runtime: x may be NULL (or a zero-length array) when
// nnz = 0, so such a product must write y = 0 with a fill kernel and launch
// no kernel that reads x.  Prints the launched kernels of each call and one
// summary line; exits 0 when every check holds.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "spmv.h"

extern "C" const char *mock_launch_log(void);

namespace {
int g_fail = 0;

void check(bool ok, const char *what) {
    if (!ok) {
        std::printf("FAIL %s (%s)\n", what, spmv_last_error());
        ++g_fail;
    }
}

// every launched kernel of the last call is the zero fill
bool only_fill(const char *what) {
    const std::string log = mock_launch_log();
    std::printf("%s launched:\n%s", what, log.c_str());
    if (log.empty()) return false;
    size_t pos = 0;
    while (pos < log.size()) {
        const size_t nl = log.find('\n', pos);
        const std::string name = log.substr(pos, nl - pos);
        if (name.find("k_fill_zero") == std::string::npos) return false;
        pos = nl + 1;
    }
    return true;
}
}  // namespace

int main() {
    // 5 x 3 scalar CSR and 4 x 2 block CSR, both without stored entries,
    // and a 5 x 0 scalar CSR (no column at all)
    const int32_t rp[6] = {0, 0, 0, 0, 0, 0};
    std::vector<double> y(64, 1.0);
    std::vector<float> y32(64, 1.0f);
    for (int n_cols : {3, 0}) {
        spmv_matrix *A = nullptr;
        check(spmv_create(5, n_cols, 0, rp, nullptr, nullptr, SPMV_VALUES_FP32 | SPMV_VALUES_BF16, nullptr, &A) ==
                  SPMV_OK, "create nnz = 0");
        if (!A) continue;
        (void)mock_launch_log();
        check(spmv_apply(A, nullptr, y.data(), nullptr) == SPMV_OK, "spmv_apply x = NULL");
        check(only_fill("spmv_apply"), "spmv_apply launches only the zero fill");
        check(spmv_apply_f32(A, nullptr, y32.data(), nullptr) == SPMV_OK, "spmv_apply_f32 x = NULL");
        check(only_fill("spmv_apply_f32"), "spmv_apply_f32 launches only the zero fill");
        check(spmv_apply_f32v(A, nullptr, y.data(), nullptr) == SPMV_OK, "spmv_apply_f32v x = NULL");
        check(only_fill("spmv_apply_f32v"), "spmv_apply_f32v launches only the zero fill");
        check(spmv_apply_bf16(A, nullptr, y32.data(), nullptr) == SPMV_OK, "spmv_apply_bf16 x = NULL");
        check(only_fill("spmv_apply_bf16"), "spmv_apply_bf16 launches only the zero fill");
        check(spmv_spmm(A, 3, nullptr, y.data(), nullptr) == SPMV_OK, "spmv_spmm X = NULL");
        check(only_fill("spmv_spmm"), "spmv_spmm launches only the zero fill");
        // y is still required
        check(spmv_apply(A, nullptr, nullptr, nullptr) == SPMV_EINVAL, "spmv_apply y = NULL rejected");
        check(spmv_destroy(A) == SPMV_OK, "destroy");
    }
    {
        const int32_t brp[5] = {0, 0, 0, 0, 0};
        spmv_matrix *B = nullptr;
        check(spmv_create_bsr3(4, 2, 0, brp, nullptr, nullptr, SPMV_VALUES_FP32, &B) == SPMV_OK, "create bsr3 nnz = 0");
        if (B) {
            (void)mock_launch_log();
            check(bsr3_spmm(B, 4, nullptr, y.data(), nullptr) == SPMV_OK, "bsr3_spmm X = NULL");
            check(only_fill("bsr3_spmm"), "bsr3_spmm launches only the zero fill");
            check(bsr3_spmm_f32(B, 1, nullptr, y32.data(), nullptr) == SPMV_OK, "bsr3_spmm_f32 X = NULL");
            check(only_fill("bsr3_spmm_f32"), "bsr3_spmm_f32 launches only the zero fill");
            check(spmv_apply(B, nullptr, y.data(), nullptr) == SPMV_OK, "spmv_apply on bsr3 x = NULL");
            check(only_fill("spmv_apply (bsr3)"), "spmv_apply on bsr3 launches only the zero fill");
            check(spmv_destroy(B) == SPMV_OK, "destroy bsr3");
        }
    }
    {
        // a matrix with entries still launches its product kernels
        const int32_t rp1[3] = {0, 1, 2};
        const int32_t ci[2] = {0, 1};
        const double va[2] = {2.0, 3.0};
        spmv_matrix *C = nullptr;
        check(spmv_create(2, 2, 2, rp1, ci, va, 0, nullptr, &C) == SPMV_OK, "create 2 x 2");
        if (C) {
            (void)mock_launch_log();
            std::vector<double> x(2, 1.0);
            check(spmv_apply(C, x.data(), y.data(), nullptr) == SPMV_OK, "spmv_apply 2 x 2");
            const std::string log = mock_launch_log();
            check(!log.empty() && log.find("k_fill_zero") == std::string::npos, "2 x 2 product launches its kernel");
            check(spmv_apply(C, nullptr, y.data(), nullptr) == SPMV_EINVAL, "x = NULL rejected when nnz > 0");
            check(spmv_destroy(C) == SPMV_OK, "destroy 2 x 2");
        }
    }
    std::printf("summary failures=%d\n", g_fail);
    return g_fail == 0 ? 0 : 1;
}
