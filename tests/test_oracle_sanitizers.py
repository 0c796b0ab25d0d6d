"""The oracle's C code under the compiler's sanitizers (CPU only).

A small driver links oracle/emd_oracle.c directly and runs every batch entry
point (explicit pairs, the labelling cross product, the pairwise triangle)
with several worker threads and with one, comparing the results bit for
bit.  It is built twice: with AddressSanitizer and UndefinedBehaviorSanitizer
(heap and stack bounds, use after free, leaks, signed overflow, bad shifts),
and with ThreadSanitizer (data races between the pthread workers).  A
sanitizer report makes the driver exit non-zero."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "emd_oracle.h"

static uint64_t st = 88172645463325252ull;
static double rnd(void) {   /* xorshift64, uniform in [0, 1) */
    st ^= st << 13; st ^= st >> 7; st ^= st << 17;
    return (double)(st >> 11) * (1.0 / 9007199254740992.0);
}

typedef struct { int64_t n; int64_t *off; double *x, *w; } set_t;

static set_t make(int64_t n, int tmax, int d, int zero_every) {
    set_t s;
    s.n = n;
    s.off = malloc(sizeof(int64_t) * (n + 1));
    s.off[0] = 0;
    for (int64_t i = 0; i < n; ++i) s.off[i + 1] = s.off[i] + 1 + (int64_t)(rnd() * tmax);
    s.x = malloc(sizeof(double) * s.off[n] * d);
    s.w = malloc(sizeof(double) * s.off[n]);
    for (int64_t a = 0; a < s.off[n] * d; ++a) s.x[a] = floor(rnd() * 6.0);   /* many ties */
    for (int64_t a = 0; a < s.off[n]; ++a) s.w[a] = (zero_every && a % zero_every == 0) ? 0.0 : 0.1 + rnd();
    return s;
}

static void drop(set_t *s) { free(s->off); free(s->x); free(s->w); }

static int same(const void *a, const void *b, size_t bytes, const char *what) {
    if (memcmp(a, b, bytes) != 0) { fprintf(stderr, "%s differs between thread counts\n", what); return 1; }
    return 0;
}

int main(void) {
    const int d = 3;
    int bad = 0;
    set_t A = make(60, 12, d, 7), B = make(9, 10, d, 0);
    /* explicit pairs, including out-of-range indices (rejected as a batch) */
    const int64_t m = 200;
    int64_t *pairs = malloc(sizeof(int64_t) * 2 * m);
    for (int64_t k = 0; k < m; ++k) { pairs[2 * k] = k % A.n; pairs[2 * k + 1] = (k * 7) % B.n; }
    double *d1 = malloc(sizeof(double) * m), *d4 = malloc(sizeof(double) * m);
    int32_t *s1 = malloc(sizeof(int32_t) * m), *s4 = malloc(sizeof(int32_t) * m);
    long long *p1 = malloc(sizeof(long long) * m), *p4 = malloc(sizeof(long long) * m);
    long long *b1 = malloc(sizeof(long long) * m), *b4 = malloc(sizeof(long long) * m);
    for (int rule = 0; rule < 2; ++rule)
        for (int ba = 0; ba < 3; ba += 2) {
            if (oracle_emd_batch(d, A.off, A.x, A.w, A.n, B.off, B.x, B.w, B.n, pairs, m, rule, ba, 1, d1, s1, p1,
                                 b1) != 0) bad |= 1;
            if (oracle_emd_batch(d, A.off, A.x, A.w, A.n, B.off, B.x, B.w, B.n, pairs, m, rule, ba, 4, d4, s4, p4,
                                 b4) != 0) bad |= 1;
            bad |= same(d1, d4, sizeof(double) * m, "emd_batch dist");
            bad |= same(s1, s4, sizeof(int32_t) * m, "emd_batch status");
            bad |= same(p1, p4, sizeof(long long) * m, "emd_batch pivots");
            bad |= same(b1, b4, sizeof(long long) * m, "emd_batch bland pivots");
        }
    pairs[7] = B.n;   /* out of range: the whole call is refused */
    if (oracle_emd_batch(d, A.off, A.x, A.w, A.n, B.off, B.x, B.w, B.n, pairs, m, 0, 0, 4, d4, s4, p4, b4) != -2)
        bad |= 1;
    /* labelling cross product */
    int32_t *l1 = malloc(sizeof(int32_t) * A.n), *l4 = malloc(sizeof(int32_t) * A.n);
    double *bst1 = malloc(sizeof(double) * A.n), *bst4 = malloc(sizeof(double) * A.n);
    double *all1 = malloc(sizeof(double) * A.n * B.n), *all4 = malloc(sizeof(double) * A.n * B.n);
    int32_t *r1 = malloc(sizeof(int32_t) * A.n), *r4 = malloc(sizeof(int32_t) * A.n);
    if (oracle_assign(d, A.off, A.x, A.w, A.n, B.off, B.x, B.w, B.n, 0, 1, l1, bst1, all1, r1, NULL, NULL) != 0)
        bad |= 1;
    if (oracle_assign(d, A.off, A.x, A.w, A.n, B.off, B.x, B.w, B.n, 0, 5, l4, bst4, all4, r4, NULL, NULL) != 0)
        bad |= 1;
    bad |= same(l1, l4, sizeof(int32_t) * A.n, "assign labels");
    bad |= same(all1, all4, sizeof(double) * A.n * B.n, "assign matrix");
    /* pairwise triangle */
    const int64_t pm = A.n * (A.n - 1) / 2;
    double *c1 = malloc(sizeof(double) * pm), *c4 = malloc(sizeof(double) * pm);
    int32_t *cs1 = malloc(sizeof(int32_t) * pm), *cs4 = malloc(sizeof(int32_t) * pm);
    if (oracle_pairwise(d, A.off, A.x, A.w, A.n, 1, 1, c1, cs1, NULL, NULL) != 0) bad |= 1;
    if (oracle_pairwise(d, A.off, A.x, A.w, A.n, 1, 6, c4, cs4, NULL, NULL) != 0) bad |= 1;
    bad |= same(c1, c4, sizeof(double) * pm, "pairwise");
    /* single solves with every output */
    double val, plan[16 * 16], u[16], v[16];
    long long piv, bl;
    for (int64_t i = 0; i < 12; ++i) {
        const int t = (int)(A.off[i + 1] - A.off[i]), s = (int)(B.off[1] - B.off[0]);
        int rc = oracle_emd_pair(t, s, d, A.x + A.off[i] * d, A.w + A.off[i], B.x, B.w, (int)(i & 1), 1, &val,
                                 plan, u, v, &piv, &bl);
        if (rc != 0 && rc != 1) bad |= 1;
    }
    free(pairs); free(d1); free(d4); free(s1); free(s4); free(p1); free(p4); free(b1); free(b4);
    free(l1); free(l4); free(bst1); free(bst4); free(all1); free(all4); free(r1); free(r4);
    free(c1); free(c4); free(cs1); free(cs4);
    drop(&A); drop(&B);
    printf(bad ? "MISMATCH\n" : "ok\n");
    return bad;
}
"""


def build_and_run(tmp_path, flags, env_extra):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", *flags, "-I", ORACLE, str(src),
           os.path.join(ORACLE, "emd_oracle.c"), "-o", str(exe), "-lm", "-pthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, **env_extra)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
    assert "Sanitizer" not in r.stderr, r.stderr


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                  {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
                   "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})


def test_oracle_worker_threads_under_thread_sanitizer(tmp_path):
    build_and_run(tmp_path, ["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"})
