// Sanitizer driver of the C ABI's host side (test infrastructure): linked
// against a build of libhaar whose host code carries AddressSanitizer and
// UndefinedBehaviorSanitizer, run by tests/test_sanitizers.py on a machine
// without a GPU.  Every call here either fails argument validation, which
// runs before any HIP call, or is host-only (depth limits, status strings,
// workspace sizes, plan creation, the tuning table and its JSON file), so
// nothing touches a device.  Exit status 0 means every call returned the
// expected code without a sanitizer report.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "haar.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
    if (got != want) {
        fprintf(stderr, "FAIL %s: got %d want %d (%s)\n", what, got, want, haar_last_error());
        ++failures;
    }
}

int main(int argc, char** argv) {
    void* X = (void*)0x10000000;
    void* Y = (void*)0x20000000;
    double* LOSS = (double*)0x30000000;
    const float thr[40] = {0};
    // plain transforms: every validation path
    expect(haar_fwd_1d(X, Y, 0, 1, 1, 0, 0), HAAR_ERR_SHAPE, "1d length 0");
    expect(haar_fwd_1d(X, Y, 64, 7, 1, 0, 0), HAAR_ERR_LEVELS, "1d levels");
    expect(haar_inv_1d(X, Y, 64, 3, 1, 9, 0), HAAR_ERR_DTYPE, "1d dtype");
    expect(haar_inv_1d(X, (char*)X + 8, 64, 3, 1, 0, 0), HAAR_ERR_ALIAS, "1d alias");
    expect(haar_fwd_1d(nullptr, Y, 64, 3, 1, 0, 0), HAAR_ERR_NULL, "1d null");
    expect(haar_fwd_1d(X, Y, 64, 3, -1, 0, 0), HAAR_ERR_SHAPE, "1d batch < 0");
    expect(haar_fwd_1d(X, Y, INT64_MAX / 2, 3, 4, 0, 0), HAAR_ERR_SHAPE, "1d overflow");
    expect(haar_fwd_2d(X, Y, 0, 8, 1, 1, 0, 0), HAAR_ERR_SHAPE, "2d height 0");
    expect(haar_fwd_2d(X, Y, INT64_MAX / 2, 8, 1, 1, 0, 0), HAAR_ERR_SHAPE, "2d overflow");
    expect(haar_inv_2d(X, Y, 8, 8, 4, 1, 0, 0), HAAR_ERR_LEVELS, "2d levels");
    expect(haar_inv_2d(X, (char*)X + 4, 8, 8, 1, 1, 0, 0), HAAR_ERR_ALIAS, "2d alias");
    expect(haar_fwd_3d(X, Y, 8, 8, 8, 4, 1, 0, 0), HAAR_ERR_LEVELS, "3d levels");
    expect(haar_inv_3d(X, Y, 1 << 30, 1 << 30, 1 << 30, 1, 1, 0, 0), HAAR_ERR_SHAPE, "3d overflow");
    expect(haar_fwd_3d(nullptr, Y, 8, 8, 8, 1, 1, 0, 0), HAAR_ERR_NULL, "3d null");
    // batch 0: nothing to do, even with NULL pointers
    expect(haar_fwd_2d(nullptr, nullptr, 8, 8, 3, 0, 1, 0), HAAR_OK, "2d batch 0");
    // fused calls
    expect(haar_shrink_1d(X, Y, 1 << 14, 13, 1, 0, 0, thr, 0), HAAR_ERR_UNSUPPORTED, "shrink1d depth");
    expect(haar_shrink_2d(X, Y, 64, 64, 2, 1, 0, 7, thr, 0), HAAR_ERR_ARG, "shrink2d mode");
    const float bad[2] = {1.0f, -1.0f};
    expect(haar_shrink_2d(X, Y, 64, 64, 2, 1, 0, 0, bad, 0), HAAR_ERR_ARG, "shrink2d threshold");
    expect(haar_shrink_2d(X, Y, 64, 64, 2, 1, 0, 0, nullptr, 0), HAAR_ERR_NULL, "shrink2d thresholds NULL");
    expect(haar_l1_grad_2d(X, Y, nullptr, 64, 64, 2, 1, 0, 0), HAAR_ERR_NULL, "l1 loss NULL");
    expect(haar_l1_grad_2d(X, Y, LOSS, 64, 64, 6, 1, 0, 0), HAAR_ERR_UNSUPPORTED, "l1 depth");
    expect(haar_l1_grad_2d_noalloc(X, Y, LOSS, 64, 64, 6, 1, 0, 0), HAAR_ERR_UNSUPPORTED, "noalloc depth");
    expect(haar_l1_grad_2d_noalloc((void*)(1ull << 40), (void*)(1ull << 42), LOSS, 32, 128, 5,
                                   (1 << 19) + 1, 0, 0),
           HAAR_ERR_WORKSPACE, "noalloc limit");
    expect(haar_direct_1d(X, Y, 64, 3, 1, 0, 0, nullptr, 0, 0), HAAR_ERR_NULL, "direct workspace NULL");
    expect(haar_direct_1d(X, Y, 64, 3, 1, 0, 0, (void*)0x40000000, 16, 0), HAAR_ERR_WORKSPACE,
           "direct workspace small");
    // host-only functions
    expect(haar_max_levels_1d(65536), 16, "max levels 1d");
    expect(haar_max_levels_2d(4096, 4097), 13, "max levels 2d");
    expect(haar_max_levels_3d(1, 1, 1), 0, "max levels 3d");
    if (haar_direct_workspace_size(65, 1) == 0) ++failures;
    for (int s = -1; s <= 12; ++s)
        if (!haar_status_string(s) || !*haar_status_string(s)) ++failures;
    if (!haar_version() || !*haar_version()) ++failures;
    // tuning table: candidates, names, forcing, JSON round trip
    for (int dt = 0; dt < 3; ++dt) {
        const int n = haar_tune_candidates_2d(dt);
        if (n < 2) ++failures;
        for (int i = -1; i <= n; ++i) (void)haar_tune_candidate_name(dt, i);
        expect(haar_force_config_2d(dt, n), HAAR_ERR_UNSUPPORTED, "force 2d out of range");
        expect(haar_force_config_2d(dt, 0), HAAR_OK, "force 2d");
        expect(haar_force_config_2d(dt, -1), HAAR_OK, "force 2d reset");
        expect(haar_force_config_1d(dt, haar_tune_candidates_1d()), HAAR_ERR_UNSUPPORTED, "force 1d range");
    }
    expect(haar_tune_2d(0, 0, 64, 64, 2, 1, nullptr, 0, 0, nullptr), HAAR_ERR_NULL, "tune2d NULL");
    if (argc > 1) {
        expect(haar_tune_save(argv[1]), HAAR_OK, "tune save");
        expect(haar_tune_load(argv[1]), HAAR_OK, "tune load");
    }
    expect(haar_tune_load("/nonexistent/dir/table.json"), HAAR_ERR_UNSUPPORTED, "tune load missing");
    // plans: creation and sizes are host work
    haar_item_2d it2[3] = {{X, Y, 37, 300, 4}, {(char*)X + (1 << 20), (char*)Y + (1 << 20), 256, 512, 5},
                           {(char*)X + (2 << 20), (char*)Y + (2 << 20), 5, 7, 2}};
    haar_plan* p = nullptr;
    expect(haar_plan_create_2d(it2, 3, 0, 0, &p), HAAR_OK, "plan2d create");
    size_t ws = 0;
    expect(haar_plan_workspace_size(p, &ws), HAAR_OK, "plan2d workspace");
    int64_t tiles = 0;
    int32_t grid = 0;
    expect(haar_plan_info(p, &tiles, &grid), HAAR_OK, "plan2d info");
    for (int c = 0; c < 10; ++c) expect(haar_plan_set_config(p, c), HAAR_OK, "plan2d config");
    expect(haar_plan_set_config(p, 10), HAAR_ERR_UNSUPPORTED, "plan2d config range");
    expect(haar_plan_execute(p, nullptr, 0), HAAR_ERR_WORKSPACE, "plan2d no workspace");
    expect(haar_plan_execute(p, (void*)0x50000000, 0), HAAR_ERR_PLAN, "plan2d not uploaded");
    expect(haar_plan_destroy(p), HAAR_OK, "plan2d destroy");
    haar_item_2d bad2 = {X, Y, 8, 8, 6};
    expect(haar_plan_create_2d(&bad2, 1, 0, 0, &p), HAAR_ERR_LEVELS, "plan2d bad item");
    haar_item_1d it1[2] = {{X, Y, 100003, 17}, {(char*)X + (1 << 20), (char*)Y + (1 << 20), 1000, 10}};
    expect(haar_plan_create_1d(it1, 2, 1, 1, &p), HAAR_OK, "plan1d create");
    expect(haar_plan_workspace_size(p, &ws), HAAR_OK, "plan1d workspace");
    expect(haar_plan_destroy(p), HAAR_OK, "plan1d destroy");
    haar_item_1d bad1 = {X, Y, 64, 7};
    expect(haar_plan_create_1d(&bad1, 1, 0, 0, &p), HAAR_ERR_LEVELS, "plan1d bad item");
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("abi sanitizer driver: all calls clean\n");
    return 0;
}
