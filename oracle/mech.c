/* Oracle mechanism reader (test infrastructure only; see oracle.h).
 * Reads the whitespace-separated text format written by the input generator. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct { FILE *fh; int err; } rd;

static int tok(rd *r, char *buf, size_t cap) {
    int c;
    for (;;) {
        c = fgetc(r->fh);
        if (c == EOF) { r->err = 1; return 0; }
        if (c == '#') { while (c != '\n' && c != EOF) c = fgetc(r->fh); continue; }
        if (c > ' ') break;
    }
    size_t n = 0;
    while (c != EOF && c > ' ') {
        if (n + 1 < cap) buf[n++] = (char)c;
        c = fgetc(r->fh);
    }
    buf[n] = 0;
    return 1;
}

static double rdd(rd *r) {
    char b[128];
    if (!tok(r, b, sizeof b)) return 0.0;
    char *e;
    double v = strtod(b, &e);
    if (*e) r->err = 1;
    return v;
}

static int rdi(rd *r) {
    char b[64];
    if (!tok(r, b, sizeof b)) return 0;
    char *e;
    long v = strtol(b, &e, 10);
    if (*e) r->err = 1;
    return (int)v;
}

static void expect(rd *r, const char *word) {
    char b[64];
    if (!tok(r, b, sizeof b) || strcmp(b, word) != 0) r->err = 1;
}

void or_mech_free(or_mech *m) {
    if (!m) return;
    if (m->rx) for (int j = 0; j < m->R; ++j) free(m->rx[j].eff);
    free(m->rx); free(m->W); free(m->comp); free(m->Tlow); free(m->Tmid); free(m->Thigh);
    free(m->alow); free(m->ahigh); free(m);
}

int or_mech_load(const char *path, or_mech **out) {
    *out = NULL;
    rd r = { fopen(path, "r"), 0 };
    if (!r.fh) return -1;
    or_mech *m = calloc(1, sizeof *m);
    char b[128];
    expect(&r, "rkmech");
    if (rdi(&r) != 1) r.err = 1;
    expect(&r, "name"); tok(&r, b, sizeof b);
    expect(&r, "elements");
    m->E = rdi(&r);
    for (int e = 0; e < m->E && !r.err; ++e) tok(&r, b, sizeof b);
    expect(&r, "species");
    m->K = rdi(&r);
    if (r.err || m->K <= 0 || m->E <= 0) goto fail;
    int K = m->K;
    m->W = calloc(K, sizeof(double)); m->comp = calloc((size_t)K * m->E, sizeof(int));
    m->Tlow = calloc(K, sizeof(double)); m->Tmid = calloc(K, sizeof(double)); m->Thigh = calloc(K, sizeof(double));
    m->alow = calloc((size_t)K * 7, sizeof(double)); m->ahigh = calloc((size_t)K * 7, sizeof(double));
    for (int k = 0; k < K && !r.err; ++k) {
        tok(&r, b, sizeof b);
        m->W[k] = rdd(&r);
        for (int e = 0; e < m->E; ++e) m->comp[k * m->E + e] = rdi(&r);
    }
    expect(&r, "thermo");
    for (int i = 0; i < K && !r.err; ++i) {
        int k = rdi(&r);
        if (k < 0 || k >= K) { r.err = 1; break; }
        m->Tlow[k] = rdd(&r); m->Tmid[k] = rdd(&r); m->Thigh[k] = rdd(&r);
        for (int a = 0; a < 7; ++a) m->alow[k * 7 + a] = rdd(&r);
        for (int a = 0; a < 7; ++a) m->ahigh[k * 7 + a] = rdd(&r);
    }
    expect(&r, "reactions");
    m->R = rdi(&r);
    if (r.err || m->R < 0) goto fail;
    m->rx = calloc(m->R > 0 ? m->R : 1, sizeof(or_reaction));
    for (int j = 0; j < m->R && !r.err; ++j) {
        or_reaction *x = &m->rx[j];
        x->kind = rdi(&r);
        x->nr = rdi(&r);
        if (x->nr < 1 || x->nr > 2) { r.err = 1; break; }
        for (int s = 0; s < x->nr; ++s) x->reac[s] = rdi(&r);
        x->np = rdi(&r);
        if (x->np < 1 || x->np > 2) { r.err = 1; break; }
        for (int s = 0; s < x->np; ++s) x->prod[s] = rdi(&r);
        x->A = rdd(&r); x->b = rdd(&r); x->Ea = rdd(&r);
        if (x->kind == 2) {
            x->A0 = rdd(&r); x->b0 = rdd(&r); x->Ea0 = rdd(&r);
            for (int t = 0; t < 4; ++t) x->troe[t] = rdd(&r);
        }
        if (x->kind == 1 || x->kind == 2) {
            x->eff = malloc(K * sizeof(double));
            for (int k = 0; k < K; ++k) x->eff[k] = 1.0;
            int ne = rdi(&r);
            for (int t = 0; t < ne && !r.err; ++t) {
                int k = rdi(&r);
                double a = rdd(&r);
                if (k < 0 || k >= K) { r.err = 1; break; }
                x->eff[k] = a;
            }
        } else if (x->kind != 0) {
            r.err = 1;
        }
        for (int s = 0; s < x->nr; ++s) if (x->reac[s] < 0 || x->reac[s] >= K) r.err = 1;
        for (int s = 0; s < x->np; ++s) if (x->prod[s] < 0 || x->prod[s] >= K) r.err = 1;
    }
    expect(&r, "end");
    if (r.err) goto fail;
    fclose(r.fh);
    *out = m;
    return 0;
fail:
    fclose(r.fh);
    or_mech_free(m);
    return -2;
}

int or_mech_dims(const or_mech *m, int *K, int *R, int *E) {
    *K = m->K; *R = m->R; *E = m->E;
    return 0;
}
