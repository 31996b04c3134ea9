/*
 * Drives the host-only entry points of libwave2d (scheme construction,
 * weights, limits, tuning tables, status strings and the argument checks
 * that run before any device work) for a build whose host code carries
 * AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_lib_sanitized.py).  No call here reaches a device: every
 * stepping call gets arguments its validation rejects.  Exit code 0 and no
 * sanitizer report means the host code stayed in bounds and defined.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "wave2d.h"

static int fails = 0, checks = 0;

static void expect(int cond, const char* what)
{
    ++checks;
    if (!cond) {
        ++fails;
        printf("FAILED: %s (%s)\n", what, wave2d_last_error());
    }
}

/* Offset of monomial exponent a under the paper's correspondence (Sec. 4,
 * eq. invMcKinney): (-1)^a floor((a + 1) / 2). */
static int q_of(int a) { return (a % 2 ? -1 : 1) * ((a + 1) / 2); }

/* The complete monomial set of degree `deg` and its node set. */
static int complete_set(int deg, int32_t* nodes, int32_t* exps)
{
    int m = 0;
    for (int d = 0; d <= deg; ++d)
        for (int a = 0; a <= d; ++a) {
            exps[2 * m] = a;
            exps[2 * m + 1] = d - a;
            nodes[2 * m] = q_of(a);
            nodes[2 * m + 1] = q_of(d - a);
            ++m;
        }
    return m;
}

int main(void)
{
    int32_t nodes[2 * 64], exps[2 * 64];
    int ids[8], nid = 0;
    double w2[9], wa[9], wb[9];

    /* complete sets of degree 1..6 (degree 2 is the 5-point set's even
     * part, degree 6 reaches three lines out) */
    for (int deg = 2; deg <= 6; ++deg) {
        const int m = complete_set(deg, nodes, exps);
        int id = -1;
        const int r = wave2d_scheme_create(m, nodes, exps, &id);
        expect(r == WAVE2D_OK && id >= 1000, "complete set accepted");
        if (r == WAVE2D_OK) ids[nid++] = id;
    }
    /* the axis "cross" set */
    {
        const int32_t cn[] = {0, 0, 1, 0, -1, 0, 0, 1, 0, -1, 2, 0, -2, 0, 0, 2, 0, -2};
        const int32_t ce[] = {0, 0, 1, 0, 0, 1, 2, 0, 0, 2, 3, 0, 0, 3, 4, 0, 0, 4};
        int id = -1;
        expect(wave2d_scheme_create(9, cn, ce, &id) == WAVE2D_OK, "cross set accepted");
        if (id >= 1000) ids[nid++] = id;
    }
    /* rejections: singular, asymmetric, weight four lines out, duplicates,
     * sizes, degree, NULL */
    {
        const int32_t sn[] = {0, 0, 1, 0, -1, 0, 0, 1, 0, -1};
        const int32_t se[] = {0, 0, 1, 0, 0, 1, 2, 0, 3, 0};
        int id;
        expect(wave2d_scheme_create(5, sn, se, &id) == WAVE2D_EINVAL, "singular rejected");
        const int32_t an[] = {0, 0, 1, 0, -1, 0, 0, 1, 1, 1};
        const int32_t ae[] = {0, 0, 1, 0, 0, 1, 2, 0, 1, 1};
        expect(wave2d_scheme_create(5, an, ae, &id) == WAVE2D_EINVAL, "asymmetric rejected");
        const int32_t fn[] = {0, 0, 1, 0, -1, 0, 0, 1, 0, -1, 2, 0, -2, 0, 0, 2, 0, -2, 4, 0, -4, 0, 0, 4, 0, -4};
        const int32_t fe[] = {0, 0, 1, 0, 0, 1, 2, 0, 0, 2, 3, 0, 0, 3, 4, 0, 0, 4, 5, 0, 0, 5, 6, 0, 0, 6};
        expect(wave2d_scheme_create(13, fn, fe, &id) == WAVE2D_EINVAL, "four lines out rejected");
        const int32_t dn[] = {0, 0, 0, 0};
        const int32_t de[] = {0, 0, 1, 0};
        expect(wave2d_scheme_create(2, dn, de, &id) == WAVE2D_EINVAL, "duplicate node rejected");
        expect(wave2d_scheme_create(0, dn, de, &id) == WAVE2D_EINVAL, "m = 0 rejected");
        expect(wave2d_scheme_create(65, nodes, exps, &id) == WAVE2D_EINVAL, "m = 65 rejected");
        expect(wave2d_scheme_create(2, dn, de, NULL) == WAVE2D_EINVAL, "NULL id rejected");
        const int32_t he[] = {0, 0, 13, 0};
        const int32_t hn[] = {0, 0, 1, 0};
        expect(wave2d_scheme_create(2, hn, he, &id) == WAVE2D_EINVAL, "degree 13 rejected");
        const int32_t on[] = {0, 0, 9, 0};
        expect(wave2d_scheme_create(2, on, de, &id) == WAVE2D_EINVAL, "node 9 steps out rejected");
    }
    /* weights and limits of every scheme */
    const int builtin[] = {WAVE2D_P5, WAVE2D_P9, WAVE2D_P13, WAVE2D_C9};
    for (int k = 0; k < 4 + nid; ++k) {
        const int s = k < 4 ? builtin[k] : ids[k - 4];
        const double lmax = wave2d_lambda_max(s);
        expect(lmax > 0.0 && lmax < 4.0, "stability limit in range");
        for (int n = 1; n <= 9; ++n) {
            const int r = wave2d_class_weights(s, 0, 0.5 * lmax, n, w2, wa, wb);
            (void)r;
        }
        expect(wave2d_class_weights(s, WAVE2D_FIRST_CONVENTIONAL, 0.5 * lmax, 9, w2, NULL, wb) == WAVE2D_OK,
               "nine-class weights");
        expect(wave2d_class_weights(s, 0, 0.5, 0, w2, wa, wb) == WAVE2D_EINVAL, "nclass 0 rejected");
        expect(wave2d_class_weights(s, 0, 0.5, 10, w2, wa, wb) == WAVE2D_EINVAL, "nclass 10 rejected");
        expect(wave2d_class_weights(s, 0, NAN, 9, w2, wa, wb) == WAVE2D_EINVAL, "NaN lambda rejected");
        (void)wave2d_weights(s, 0, 0.3, w2, wa, wb);
    }
    expect(wave2d_lambda_max(4242) < 0.0, "unknown scheme has no limit");
    expect(wave2d_weights(4242, 0, 0.3, w2, wa, wb) == WAVE2D_EINVAL, "unknown scheme weights rejected");

    /* tuning tables (host only) */
    wave2d_tuning t = {6, 40}, g;
    expect(wave2d_set_tuning(WAVE2D_F32C, WAVE2D_P9, &t) == WAVE2D_OK, "tuning set");
    expect(wave2d_get_tuning(WAVE2D_F32C, WAVE2D_P9, 1000, 1000, &g) == WAVE2D_OK && g.depth == 6, "tuning read");
    expect(wave2d_set_tuning(WAVE2D_F32C, WAVE2D_P9, NULL) == WAVE2D_OK, "tuning reset");
    t.depth = 5;
    expect(wave2d_set_tuning(WAVE2D_F64, WAVE2D_P5, &t) == WAVE2D_EINVAL, "depth 5 rejected");
    expect(wave2d_set_tuning(7, WAVE2D_P5, NULL) == WAVE2D_EINVAL, "precision 7 rejected");
    if (nid > 4) expect(wave2d_get_tuning(WAVE2D_F32C, ids[4], 64, 64, &g) == WAVE2D_EINVAL, "wide scheme has no tuning");

    /* sizes and strings */
    expect(wave2d_work_bytes(WAVE2D_F32C, 100, 100, 128) > 0, "work bytes");
    expect(wave2d_work_bytes(WAVE2D_F32C, 100, 100, 50) == 0, "ld < nx has no size");
    expect(wave2d_work_bytes(9, 100, 100, 100) == 0, "unknown precision has no size");
    for (int st = -8; st <= 1; ++st) expect(strlen(wave2d_status_str(st)) > 0, "status string");

    /* stepping calls whose validation fails before any device work */
    double d8[16];
    float f4[16];
    expect(wave2d_first_step(2, 5, 5, 0.1, 0.05, 1.0, WAVE2D_P5, 0, d8, d8, d8, NULL) == WAVE2D_EINVAL, "2 x 5 rejected");
    expect(wave2d_step(5, 5, 4, 0.1, 0.05, 1.0, WAVE2D_P5, 0, 1, d8, d8, NULL, 0, NULL) == WAVE2D_EINVAL, "ld < nx rejected");
    expect(wave2d_run(5, 5, 5, 0.1, 0.2, 1.0, WAVE2D_P9, 0, 3, d8, d8, d8, d8, NULL, 0, NULL) == WAVE2D_EUNSTABLE,
           "unstable Courant number rejected");
    expect(wave2d_run(5, 5, 5, 0.1, 0.05, 1.0, WAVE2D_P9, 0x80000000u, 3, d8, d8, d8, d8, NULL, 0, NULL) == WAVE2D_EINVAL,
           "unknown flag rejected");
    expect(wave2d_f32c_step(5, 5, 5, 0.1, 0.05, 1.0, WAVE2D_P13, 0, -1, f4, f4, f4, NULL, 0, NULL) == WAVE2D_EINVAL,
           "negative steps rejected");
    expect(wave2d_f32c_run(6, 6, 6, 0.1, 0.05, 1.0, WAVE2D_P13, 0, 0, d8, d8, f4, f4, f4, NULL, 0, NULL) == WAVE2D_EINVAL,
           "zero steps rejected");
    expect(wave2d_f32c_step(5, 5, 5, 0.1, 0.05, 1.0, WAVE2D_P13, WAVE2D_PERIODIC, 1, f4, f4, f4, NULL, 0, NULL) == WAVE2D_EINVAL,
           "aliased arrays rejected");
    if (nid > 4)
        expect(wave2d_run(6, 6, 6, 0.1, 0.01, 1.0, ids[4], WAVE2D_PERIODIC, 3, d8, d8, d8, d8, NULL, 0, NULL) == WAVE2D_EINVAL,
               "6 x 6 periodic wide scheme rejected");
    expect(wave2d_first_step(5, 5, 5, NAN, 0.05, 1.0, WAVE2D_P5, 0, d8, d8, d8, NULL) == WAVE2D_EINVAL, "NaN h rejected");
    expect(wave2d_norms(0, 5, 5, d8, d8, w2, NULL) == WAVE2D_EINVAL, "empty norms rejected");
    expect(wave2d_batch_create(NULL, 1, 0, NULL) == WAVE2D_EINVAL, "NULL batch output rejected");
    wave2d_batch* bt = NULL;
    expect(wave2d_batch_create(NULL, 0, 0, &bt) == WAVE2D_EINVAL, "empty batch rejected");
    expect(wave2d_batch_set_rows_cap(NULL, 64, NULL) == WAVE2D_EINVAL, "NULL batch rejected");

    printf("host entry points exercised: %d checks, %d failed\n", checks, fails);
    return fails ? 1 : 0;
}
