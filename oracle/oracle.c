/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * What it computes, for every shot independently:
 *   1. the draw u(seed, shot, l) = Philox4x32-10(ctr, key)[l mod 4] with
 *      ctr = (floor(l/4), shot mod 2^32, floor(shot/2^32), 0) and
 *      key = (seed mod 2^32, floor(seed/2^32))   [Salmon et al., SC'11];
 *   2. for each noise location, the Pauli picked by u through exact integer
 *      thresholds (the symbol laws of Section 3.1: an X-error fires with
 *      probability p, depolarizing picks each non-identity Pauli with p/3,
 *      the two-qubit one each of 15 with p/15);
 *   3. the concrete Aaronson-Gottesman tableau (Section 2.2, Eq. 1) run over
 *      the circuit, with faults applied by the Pauli-gate phase rules of
 *      Fact 1 and a random measurement taking its outcome from bit 0 of the
 *      code (code = 1 iff u < 2^31);
 *   4. the recorded outcomes packed 64 shots per word, measurement-major,
 *      the column layout of the sample matrix of Eq. 4.
 *
 * Reset R is read as: measure (outcome random or determined, as above), then
 * apply X when the outcome is 1.  MR is M followed by that conditional X.
 * "CX/CY/CZ rec[-k] q" applies X/Y/Z to q when the k-th most recent recorded
 * outcome of this shot is 1 (the conditional Paulis of the conclusion).
 * Detector and observable outputs are XORs of this shot's recorded outcomes.
 *
 * Nothing here is blocked, fused or reordered: one shot is one pass of the
 * textbook algorithm.  Threads only split independent shots.
 */
#include "oracle.h"

#include <ctype.h>
#include <pthread.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------ */
/* errors                                                              */
/* ------------------------------------------------------------------ */

static __thread char g_err[512];

static int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

const char* oracle_last_error(void) { return g_err; }

/* ------------------------------------------------------------------ */
/* circuit                                                             */
/* ------------------------------------------------------------------ */

enum {
  OP_H, OP_S, OP_X, OP_Y, OP_Z, OP_CX, OP_M, OP_R, OP_MR,
  OP_XERR, OP_YERR, OP_ZERR, OP_DEP1, OP_DEP2, OP_TICK,
  OP_CY, OP_CZ,       /* parsed names; only record-controlled pairs are kept */
  OP_FX, OP_FY, OP_FZ, /* Pauli on a qubit if a recorded outcome is 1: (record, qubit) pairs */
  OP_DET, OP_OBS       /* detector: records; observable: index, then records */
};

typedef struct {
  int kind;
  int ntargets;
  int* targets;
  /* channel probability p = num/den and its thresholds (noise ops only) */
  int m;           /* number of non-identity outcomes */
  uint64_t T[16];  /* T[1..m]; T[m] may be 2^32 */
  char ptext[64];
} op_t;

struct oracle_circuit {
  int nq;
  int nops;
  op_t* ops;
  int nlocs;
  int nmeas;
  int ndet, nobs;  /* detectors, observables (1 + largest index) */
  int* loc_kind;   /* ORACLE_LOC_* per location */
};

typedef unsigned __int128 u128;

/* Exact decimal literal -> num/den.  Accepts [digits][.digits][e[+-]digits]. */
static int parse_decimal(const char* s, u128* num, u128* den) {
  const char* p = s;
  u128 mant = 0;
  int ndig = 0, frac = 0, seen_dot = 0, any = 0;
  while (*p) {
    if (isdigit((unsigned char)*p)) {
      if (mant != 0 || *p != '0') ndig++;
      if (ndig > 19) return -1;
      mant = mant * 10 + (u128)(*p - '0');
      if (seen_dot) frac++;
      any = 1;
      p++;
    } else if (*p == '.' && !seen_dot) {
      seen_dot = 1;
      p++;
    } else {
      break;
    }
  }
  if (!any) return -1;
  int ex = 0;
  if (*p == 'e' || *p == 'E') {
    p++;
    int sign = 1;
    if (*p == '+') p++;
    else if (*p == '-') { sign = -1; p++; }
    if (!isdigit((unsigned char)*p)) return -1;
    while (isdigit((unsigned char)*p)) {
      ex = ex * 10 + (*p - '0');
      if (ex > 60) return -1;
      p++;
    }
    ex *= sign;
  }
  if (*p != 0) return -1;
  int e10 = ex - frac;
  u128 d = 1;
  if (e10 >= 0) {
    for (int i = 0; i < e10; i++) {
      mant *= 10;
      if (mant > ((u128)1 << 100)) return -1;
    }
  } else {
    if (-e10 > 30) return -1;
    for (int i = 0; i < -e10; i++) d *= 10;
  }
  *num = mant;
  *den = d;
  return 0;
}

/* T_k = floor(k * p * 2^32 / m), p = num/den, computed exactly. */
static int compute_thresholds(const char* ptext, int m, uint64_t* T) {
  u128 num, den;
  if (parse_decimal(ptext, &num, &den) != 0)
    return fail(-2, "bad probability literal '%s'", ptext);
  if (num > den) return fail(-2, "probability %s exceeds 1", ptext);
  T[0] = 0;
  for (int k = 1; k <= m; k++) {
    u128 t = ((u128)k * num << 32) / (den * (u128)m);
    T[k] = (uint64_t)t;
  }
  return 0;
}

int oracle_thresholds(const char* p_text, int m, uint64_t* T) {
  if (!p_text || !T || m < 1 || m > 15) return fail(-1, "bad arguments");
  uint64_t tmp[16];
  int rc = compute_thresholds(p_text, m, tmp);
  if (rc) return rc;
  for (int k = 1; k <= m; k++) T[k - 1] = tmp[k];
  return 0;
}

static const struct { const char* name; int kind; int has_p; int m; } k_names[] = {
  {"H", OP_H, 0, 0},        {"S", OP_S, 0, 0},        {"X", OP_X, 0, 0},
  {"Y", OP_Y, 0, 0},        {"Z", OP_Z, 0, 0},        {"CX", OP_CX, 0, 0},
  {"CNOT", OP_CX, 0, 0},    {"M", OP_M, 0, 0},        {"R", OP_R, 0, 0},
  {"MR", OP_MR, 0, 0},      {"X_ERROR", OP_XERR, 1, 1}, {"Y_ERROR", OP_YERR, 1, 1},
  {"Z_ERROR", OP_ZERR, 1, 1}, {"DEPOLARIZE1", OP_DEP1, 1, 3},
  {"DEPOLARIZE2", OP_DEP2, 1, 15}, {"TICK", OP_TICK, 0, 0},
  {"CY", OP_CY, 0, 0},      {"CZ", OP_CZ, 0, 0},
  {"DETECTOR", OP_DET, 2, 0}, {"OBSERVABLE_INCLUDE", OP_OBS, 3, 0},
};

void oracle_free(oracle_circuit* c) {
  if (!c) return;
  for (int i = 0; i < c->nops; i++) free(c->ops[i].targets);
  free(c->ops);
  free(c->loc_kind);
  free(c);
}

int oracle_parse(const char* text, size_t len, oracle_circuit** out) {
  if (!text || !out) return fail(-1, "null argument");
  *out = NULL;
  oracle_circuit* c = calloc(1, sizeof *c);
  int cap = 64;
  c->ops = calloc(cap, sizeof(op_t));
  char* buf = malloc(len + 1);
  memcpy(buf, text, len);
  buf[len] = 0;
  int rc = 0, lineno = 0;
  long nmeas_so_far = 0;
  char* save = NULL;
  for (char* line = strtok_r(buf, "\n", &save); line; line = strtok_r(NULL, "\n", &save)) {
    lineno++;
    char* hash = strchr(line, '#');
    if (hash) *hash = 0;
    /* head: NAME or NAME(argument); the argument may contain spaces */
    char* p = line;
    while (*p == ' ' || *p == '\t' || *p == '\r') p++;
    if (!*p) continue;
    char name[64], ptext[64];
    ptext[0] = 0;
    int has_arg = 0;
    size_t nl = 0;
    while (p[nl] && (isalnum((unsigned char)p[nl]) || p[nl] == '_')) nl++;
    if (nl == 0 || nl >= sizeof name) { rc = fail(-2, "line %d: malformed instruction", lineno); break; }
    memcpy(name, p, nl);
    name[nl] = 0;
    p += nl;
    if (*p == '(') {
      char* close = strchr(p, ')');
      if (!close || (size_t)(close - p - 1) >= sizeof ptext) { rc = fail(-2, "line %d: malformed '%s('", lineno, name); break; }
      memcpy(ptext, p + 1, (size_t)(close - p - 1));
      ptext[close - p - 1] = 0;
      has_arg = 1;
      p = close + 1;
    }
    if (*p && *p != ' ' && *p != '\t' && *p != '\r') { rc = fail(-2, "line %d: malformed instruction", lineno); break; }
    int kind = -1, argk = 0, m = 0;
    for (size_t i = 0; i < sizeof k_names / sizeof k_names[0]; i++)
      if (strcmp(name, k_names[i].name) == 0) {
        kind = k_names[i].kind; argk = k_names[i].has_p; m = k_names[i].m;
      }
    if (kind < 0) { rc = fail(-3, "line %d: unsupported instruction '%s'", lineno, name); break; }
    /* argk: 0 none, 1 probability, 2 optional and ignored, 3 required index */
    if ((argk == 1 || argk == 3) && !has_arg) { rc = fail(-2, "line %d: missing argument for '%s'", lineno, name); break; }
    if (argk == 0 && has_arg) { rc = fail(-2, "line %d: argument not allowed for '%s'", lineno, name); break; }
    if (c->nops == cap) {
      cap *= 2;
      c->ops = realloc(c->ops, cap * sizeof(op_t));
    }
    op_t* op = &c->ops[c->nops];
    memset(op, 0, sizeof *op);
    op->kind = kind;
    op->m = m;
    if (argk == 1) {
      strcpy(op->ptext, ptext);
      if ((rc = compute_thresholds(ptext, m, op->T)) != 0) {
        char msg[256];
        memcpy(msg, g_err, sizeof msg - 1);
        msg[sizeof msg - 1] = 0;
        rc = fail(rc, "line %d: %s", lineno, msg);
        break;
      }
    }
    int tcap = 8;
    op->targets = malloc(tcap * sizeof(int));
    int* isrec = malloc(tcap * sizeof(int));
    if (argk == 3) {
      char* end = NULL;
      long v = strtol(ptext, &end, 10);
      if (!isdigit((unsigned char)ptext[0]) || *end != 0 || v < 0 || v > 1000000) {
        rc = fail(-2, "line %d: bad observable index '%s'", lineno, ptext);
        c->nops++;
        free(isrec);
        break;
      }
      op->targets[op->ntargets] = (int)v;
      isrec[op->ntargets++] = 0;
      if ((int)v + 1 > c->nobs) c->nobs = (int)v + 1;
    }
    char* tokp = NULL;
    for (char* t = strtok_r(p, " \t\r", &tokp); t; t = strtok_r(NULL, " \t\r", &tokp)) {
      long v;
      int rec = 0;
      char* end = NULL;
      if (strncmp(t, "rec[-", 5) == 0) {
        v = strtol(t + 5, &end, 10);
        if (!isdigit((unsigned char)t[5]) || strcmp(end, "]") != 0 || v < 1 || v > nmeas_so_far) {
          rc = fail(-2, "line %d: bad record target '%s'", lineno, t);
          break;
        }
        v = nmeas_so_far - v;   /* absolute index of the recorded outcome */
        rec = 1;
      } else {
        v = strtol(t, &end, 10);
        if (!isdigit((unsigned char)t[0]) || *end != 0 || v < 0 || v > 1000000) {
          rc = fail(-2, "line %d: bad target '%s'", lineno, t);
          break;
        }
      }
      if (op->ntargets == tcap) {
        tcap *= 2;
        op->targets = realloc(op->targets, tcap * sizeof(int));
        isrec = realloc(isrec, tcap * sizeof(int));
      }
      isrec[op->ntargets] = rec;
      op->targets[op->ntargets++] = (int)v;
      if (!rec && (int)v + 1 > c->nq) c->nq = (int)v + 1;
    }
    c->nops++;
    if (rc) { free(isrec); break; }
    /* target kinds per instruction */
    if (kind == OP_DET || kind == OP_OBS) {
      for (int i = (kind == OP_OBS); i < op->ntargets; i++)
        if (!isrec[i]) { rc = fail(-2, "line %d: '%s' takes record targets", lineno, name); break; }
      if (kind == OP_DET) c->ndet++;
    } else if (kind == OP_CX || kind == OP_CY || kind == OP_CZ) {
      if (op->ntargets % 2) rc = fail(-2, "line %d: odd number of targets", lineno);
      for (int i = 0; !rc && i < op->ntargets; i += 2) {
        if (isrec[i + 1]) rc = fail(-2, "line %d: record as the target of a pair", lineno);
        else if (!isrec[i] && kind != OP_CX) rc = fail(-3, "line %d: quantum '%s' not supported", lineno, name);
        else if (!isrec[i] && op->targets[i] == op->targets[i + 1]) rc = fail(-2, "line %d: pair on one qubit", lineno);
      }
      /* one op per pair, in order: CNOT or the controlled Pauli */
      if (!rc) {
        int np = op->ntargets / 2;
        int* tg = op->targets;
        int* rc_of = isrec;
        c->nops--;   /* the parsed op is replaced by one op per pair */
        for (int i = 0; i < np; i++) {
          if (c->nops == cap) {
            cap *= 2;
            c->ops = realloc(c->ops, cap * sizeof(op_t));
          }
          op_t* po = &c->ops[c->nops++];
          memset(po, 0, sizeof *po);
          po->kind = rc_of[2 * i] ? (kind == OP_CX ? OP_FX : kind == OP_CY ? OP_FY : OP_FZ) : OP_CX;
          po->ntargets = 2;
          po->targets = malloc(2 * sizeof(int));
          po->targets[0] = tg[2 * i];
          po->targets[1] = tg[2 * i + 1];
        }
        free(tg);
      }
    } else {
      for (int i = 0; i < op->ntargets; i++)
        if (isrec[i]) { rc = fail(-2, "line %d: '%s' takes qubit targets", lineno, name); break; }
    }
    free(isrec);
    if (rc) break;
    if (kind == OP_M || kind == OP_MR) nmeas_so_far += op->ntargets;
    if (kind == OP_TICK && op->ntargets) { rc = fail(-2, "line %d: TICK takes no targets", lineno); break; }
    if (kind == OP_DEP2) {
      if (op->ntargets % 2) { rc = fail(-2, "line %d: odd number of targets", lineno); break; }
      for (int i = 0; i < op->ntargets; i += 2)
        if (op->targets[i] == op->targets[i + 1]) { rc = fail(-2, "line %d: pair on one qubit", lineno); break; }
      if (rc) break;
    }
  }
  free(buf);
  if (rc) { oracle_free(c); return rc; }

  /* Locations in program order: each target of a 1-qubit channel, each
   * pair of DEPOLARIZE2, each target of M, R, MR. */
  int nl = 0, nm = 0;
  for (int i = 0; i < c->nops; i++) {
    op_t* op = &c->ops[i];
    switch (op->kind) {
      case OP_XERR: case OP_YERR: case OP_ZERR: case OP_DEP1: case OP_R:
        nl += op->ntargets; break;
      case OP_DEP2: nl += op->ntargets / 2; break;
      case OP_M: case OP_MR: nl += op->ntargets; nm += op->ntargets; break;
      default: break;
    }
  }
  c->nlocs = nl;
  c->nmeas = nm;
  c->loc_kind = malloc((nl ? nl : 1) * sizeof(int));
  int l = 0;
  for (int i = 0; i < c->nops; i++) {
    op_t* op = &c->ops[i];
    int k = 0, cnt = op->ntargets;
    switch (op->kind) {
      case OP_XERR: k = ORACLE_LOC_X_ERROR; break;
      case OP_YERR: k = ORACLE_LOC_Y_ERROR; break;
      case OP_ZERR: k = ORACLE_LOC_Z_ERROR; break;
      case OP_DEP1: k = ORACLE_LOC_DEPOLARIZE1; break;
      case OP_DEP2: k = ORACLE_LOC_DEPOLARIZE2; cnt /= 2; break;
      case OP_M: k = ORACLE_LOC_M; break;
      case OP_R: k = ORACLE_LOC_R; break;
      case OP_MR: k = ORACLE_LOC_MR; break;
      default: cnt = 0;
    }
    for (int j = 0; j < cnt; j++) c->loc_kind[l++] = k;
  }
  *out = c;
  return 0;
}

int oracle_dims(const oracle_circuit* c, int* n_qubits, int* n_locs, int* n_meas) {
  if (!c) return fail(-1, "null circuit");
  if (n_qubits) *n_qubits = c->nq;
  if (n_locs) *n_locs = c->nlocs;
  if (n_meas) *n_meas = c->nmeas;
  return 0;
}

int oracle_location_kinds(const oracle_circuit* c, int* kinds) {
  if (!c || !kinds) return fail(-1, "null argument");
  memcpy(kinds, c->loc_kind, (size_t)c->nlocs * sizeof(int));
  return 0;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                   */
/* ------------------------------------------------------------------ */
/* Ten rounds of: multiply words 0 and 2 by the two round multipliers,
 * keep the 64-bit products; the new words are
 *   (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0));
 * between rounds the key is advanced by the Weyl constants. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

uint32_t oracle_draw(uint64_t seed, uint64_t shot, uint64_t loc) {
  uint32_t ctr[4] = {(uint32_t)(loc >> 2), (uint32_t)shot, (uint32_t)(shot >> 32), 0};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  oracle_philox4x32_10(ctr, key, out);
  return out[loc & 3];
}

/* Code of a channel with thresholds T[1..m]: smallest k with u < T_k, else 0. */
static int code_from_draw(const op_t* op, uint32_t u) {
  for (int k = 1; k <= op->m; k++)
    if ((uint64_t)u < op->T[k]) return k;
  return 0;
}

int oracle_draw_codes(const oracle_circuit* c, uint64_t seed, uint64_t shot, uint8_t* codes) {
  if (!c || !codes) return fail(-1, "null argument");
  int l = 0;
  for (int i = 0; i < c->nops; i++) {
    const op_t* op = &c->ops[i];
    int cnt = 0;
    switch (op->kind) {
      case OP_XERR: case OP_YERR: case OP_ZERR: case OP_DEP1: cnt = op->ntargets; break;
      case OP_DEP2: cnt = op->ntargets / 2; break;
      case OP_M: case OP_R: case OP_MR: cnt = op->ntargets; break;
      default: break;
    }
    for (int j = 0; j < cnt; j++, l++) {
      uint32_t u = oracle_draw(seed, shot, (uint64_t)l);
      if (op->kind == OP_M || op->kind == OP_R || op->kind == OP_MR)
        codes[l] = (u < 0x80000000u) ? 1 : 0;
      else
        codes[l] = (uint8_t)code_from_draw(op, u);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Aaronson-Gottesman tableau (Section 2.2, Eq. 1)                     */
/* ------------------------------------------------------------------ */
/* Rows 0..n-1 destabilizers, n..2n-1 stabilizers, 2n scratch.
 * Row i holds bits x_ij, z_ij (qubit j) packed 64 per word, and phase r_i. */
typedef struct {
  int n, nw;
  uint64_t* x;
  uint64_t* z;
  uint8_t* r;
} tab_t;

static inline int getb(const uint64_t* row, int j) { return (int)((row[j >> 6] >> (j & 63)) & 1u); }
static inline void flipb(uint64_t* row, int j) { row[j >> 6] ^= (uint64_t)1 << (j & 63); }
static inline void setb(uint64_t* row, int j, int v) {
  uint64_t m = (uint64_t)1 << (j & 63);
  if (v) row[j >> 6] |= m; else row[j >> 6] &= ~m;
}
#define XR(t, i) ((t)->x + (size_t)(i) * (t)->nw)
#define ZR(t, i) ((t)->z + (size_t)(i) * (t)->nw)

static void tab_alloc(tab_t* t, int n) {
  t->n = n;
  t->nw = (n + 63) / 64;
  if (t->nw == 0) t->nw = 1;
  size_t words = (size_t)(2 * n + 1) * t->nw;
  t->x = calloc(words, 8);
  t->z = calloc(words, 8);
  t->r = calloc((size_t)(2 * n + 1), 1);
}
static void tab_free(tab_t* t) { free(t->x); free(t->z); free(t->r); }

/* |0...0>: destabilizer i = X_i, stabilizer i = Z_i, all phases +. */
static void tab_reset_all(tab_t* t) {
  size_t words = (size_t)(2 * t->n + 1) * t->nw;
  memset(t->x, 0, words * 8);
  memset(t->z, 0, words * 8);
  memset(t->r, 0, (size_t)(2 * t->n + 1));
  for (int i = 0; i < t->n; i++) {
    setb(XR(t, i), i, 1);
    setb(ZR(t, i + t->n), i, 1);
  }
}

/* H on qubit a: r ^= x z, swap x and z (the rule printed in Section 2.2). */
static void gate_h(tab_t* t, int a) {
  for (int i = 0; i < 2 * t->n; i++) {
    int x = getb(XR(t, i), a), z = getb(ZR(t, i), a);
    t->r[i] ^= (uint8_t)(x & z);
    setb(XR(t, i), a, z);
    setb(ZR(t, i), a, x);
  }
}

/* S on qubit a: r ^= x z, z ^= x. */
static void gate_s(tab_t* t, int a) {
  for (int i = 0; i < 2 * t->n; i++) {
    int x = getb(XR(t, i), a), z = getb(ZR(t, i), a);
    t->r[i] ^= (uint8_t)(x & z);
    setb(ZR(t, i), a, z ^ x);
  }
}

/* CNOT control a, target b: r ^= x_a z_b (x_b ^ z_a ^ 1); x_b ^= x_a; z_a ^= z_b. */
static void gate_cx(tab_t* t, int a, int b) {
  for (int i = 0; i < 2 * t->n; i++) {
    int xa = getb(XR(t, i), a), za = getb(ZR(t, i), a);
    int xb = getb(XR(t, i), b), zb = getb(ZR(t, i), b);
    t->r[i] ^= (uint8_t)(xa & zb & (xb ^ za ^ 1));
    setb(XR(t, i), b, xb ^ xa);
    setb(ZR(t, i), a, za ^ zb);
  }
}

/* Pauli X^px Z^pz on qubit a, Fact 1: X flips rows with z_a=1, Z rows with
 * x_a=1 (Y = both). */
static void gate_pauli(tab_t* t, int a, int px, int pz) {
  for (int i = 0; i < 2 * t->n; i++) {
    int x = getb(XR(t, i), a), z = getb(ZR(t, i), a);
    t->r[i] ^= (uint8_t)((px & z) ^ (pz & x));
  }
}

/* g(x1,z1,x2,z2): exponent of i picked up when the single-qubit Pauli
 * (x1,z1) multiplies (x2,z2).  Word-parallel: positions contributing +1 and
 * -1, from the case table
 *   (x1,z1)=(1,1) Y: z2 - x2;  (1,0) X: z2 (2 x2 - 1);  (0,1) Z: x2 (1 - 2 z2). */
static inline void g_masks(uint64_t x1, uint64_t z1, uint64_t x2, uint64_t z2,
                           uint64_t* plus, uint64_t* minus) {
  uint64_t X1 = x1 & ~z1, Z1 = ~x1 & z1, Y1 = x1 & z1;
  *plus = (X1 & x2 & z2) | (Z1 & x2 & ~z2) | (Y1 & ~x2 & z2);
  *minus = (X1 & ~x2 & z2) | (Z1 & x2 & z2) | (Y1 & x2 & ~z2);
}

/* rowsum(h, i): row h <- row i * row h; r_h from 2 r_h + 2 r_i + sum g mod 4. */
static void rowsum(tab_t* t, int h, int i) {
  long long sum = 2 * (long long)t->r[h] + 2 * (long long)t->r[i];
  uint64_t *xh = XR(t, h), *zh = ZR(t, h), *xi = XR(t, i), *zi = ZR(t, i);
  for (int w = 0; w < t->nw; w++) {
    uint64_t plus, minus;
    g_masks(xi[w], zi[w], xh[w], zh[w], &plus, &minus);
    sum += __builtin_popcountll(plus) - __builtin_popcountll(minus);
    xh[w] ^= xi[w];
    zh[w] ^= zi[w];
  }
  int m = (int)(((sum % 4) + 4) % 4);
  t->r[h] = (uint8_t)(m == 2 ? 1 : 0);
}

/* Z-basis measurement of qubit a.  If some stabilizer has x_a = 1 the
 * outcome is random and equals `random_bit`; otherwise it is determined by
 * the stabilizers.  *was_random reports which case occurred. */
static int measure(tab_t* t, int a, int random_bit, int* was_random) {
  int n = t->n, p = -1;
  for (int i = n; i < 2 * n; i++)
    if (getb(XR(t, i), a)) { p = i; break; }
  if (p >= 0) {
    for (int i = 0; i < 2 * n; i++)
      if (i != p && getb(XR(t, i), a)) rowsum(t, i, p);
    memcpy(XR(t, p - n), XR(t, p), (size_t)t->nw * 8);
    memcpy(ZR(t, p - n), ZR(t, p), (size_t)t->nw * 8);
    t->r[p - n] = t->r[p];
    memset(XR(t, p), 0, (size_t)t->nw * 8);
    memset(ZR(t, p), 0, (size_t)t->nw * 8);
    setb(ZR(t, p), a, 1);
    t->r[p] = (uint8_t)(random_bit & 1);
    *was_random = 1;
    return random_bit & 1;
  }
  int s = 2 * n;
  memset(XR(t, s), 0, (size_t)t->nw * 8);
  memset(ZR(t, s), 0, (size_t)t->nw * 8);
  t->r[s] = 0;
  for (int i = 0; i < n; i++)
    if (getb(XR(t, i), a)) rowsum(t, s, i + n);
  *was_random = 0;
  return t->r[s];
}

/* Symplectic relations of the A-G tableau: destabilizer i anticommutes with
 * stabilizer i and commutes with every other row; stabilizers commute. */
static int check_relations(const tab_t* t) {
  int n = t->n;
  for (int i = 0; i < 2 * n; i++)
    for (int j = i + 1; j < 2 * n; j++) {
      int par = 0;
      const uint64_t *xi = t->x + (size_t)i * t->nw, *zi = t->z + (size_t)i * t->nw;
      const uint64_t *xj = t->x + (size_t)j * t->nw, *zj = t->z + (size_t)j * t->nw;
      for (int w = 0; w < t->nw; w++) par ^= __builtin_popcountll((xi[w] & zj[w]) ^ (zi[w] & xj[w])) & 1;
      int want = (j == i + n) ? 1 : 0;
      if (par != want) return -1;
    }
  return 0;
}

/* ------------------------------------------------------------------ */
/* one shot                                                            */
/* ------------------------------------------------------------------ */

/* Code provider: explicit array, or draws from (seed, shot). */
typedef struct {
  const uint8_t* codes;
  uint64_t seed, shot;
} codesrc_t;

static inline int get_code(const codesrc_t* src, const op_t* op, int l) {
  if (src->codes) return src->codes[l];
  uint32_t u = oracle_draw(src->seed, src->shot, (uint64_t)l);
  if (op->kind == OP_M || op->kind == OP_R || op->kind == OP_MR) return u < 0x80000000u ? 1 : 0;
  return code_from_draw(op, u);
}

static int run_shot(const oracle_circuit* c, tab_t* t, const codesrc_t* src, uint8_t* outcomes,
                    uint8_t* was_random, int check) {
  tab_reset_all(t);
  int l = 0, k = 0;
  for (int oi = 0; oi < c->nops; oi++) {
    const op_t* op = &c->ops[oi];
    const int* q = op->targets;
    switch (op->kind) {
      case OP_H: for (int j = 0; j < op->ntargets; j++) gate_h(t, q[j]); break;
      case OP_S: for (int j = 0; j < op->ntargets; j++) gate_s(t, q[j]); break;
      case OP_X: for (int j = 0; j < op->ntargets; j++) gate_pauli(t, q[j], 1, 0); break;
      case OP_Y: for (int j = 0; j < op->ntargets; j++) gate_pauli(t, q[j], 1, 1); break;
      case OP_Z: for (int j = 0; j < op->ntargets; j++) gate_pauli(t, q[j], 0, 1); break;
      case OP_CX: for (int j = 0; j < op->ntargets; j += 2) gate_cx(t, q[j], q[j + 1]); break;
      case OP_XERR: case OP_YERR: case OP_ZERR:
        for (int j = 0; j < op->ntargets; j++, l++) {
          if (get_code(src, op, l) & 1)
            gate_pauli(t, q[j], op->kind != OP_ZERR, op->kind != OP_XERR);
        }
        break;
      case OP_DEP1:
        for (int j = 0; j < op->ntargets; j++, l++) {
          int code = get_code(src, op, l);
          if (code) gate_pauli(t, q[j], code & 1, (code >> 1) & 1);
        }
        break;
      case OP_DEP2:
        for (int j = 0; j < op->ntargets; j += 2, l++) {
          int code = get_code(src, op, l);
          if (code & 3) gate_pauli(t, q[j], code & 1, (code >> 1) & 1);
          if (code & 12) gate_pauli(t, q[j + 1], (code >> 2) & 1, (code >> 3) & 1);
        }
        break;
      case OP_M: case OP_MR: case OP_R:
        for (int j = 0; j < op->ntargets; j++, l++) {
          int rnd = 0;
          /* measure() uses the bit only when the outcome is random. */
          int bit = get_code(src, op, l) & 1;
          int m = measure(t, q[j], bit, &rnd);
          if (was_random) was_random[l] = (uint8_t)rnd;
          if (op->kind != OP_R) outcomes[k++] = (uint8_t)m;
          if (op->kind != OP_M && m) gate_pauli(t, q[j], 1, 0);
        }
        break;
      case OP_FX: case OP_FY: case OP_FZ:
        for (int j = 0; j < op->ntargets; j += 2)
          if (outcomes[q[j]]) gate_pauli(t, q[j + 1], op->kind != OP_FZ, op->kind != OP_FX);
        break;
      case OP_TICK: case OP_DET: case OP_OBS: case OP_CY: case OP_CZ: break;
    }
    if (check && check_relations(t) != 0)
      return fail(-5, "tableau relations violated after instruction %d", oi);
  }
  return 0;
}

int oracle_run_codes(const oracle_circuit* c, const uint8_t* codes, uint8_t* outcomes,
                     uint8_t* was_random, int check_invariants) {
  if (!c || !codes || !outcomes) return fail(-1, "null argument");
  tab_t t;
  tab_alloc(&t, c->nq);
  codesrc_t src = {codes, 0, 0};
  if (was_random) memset(was_random, 0, (size_t)c->nlocs);
  int rc = run_shot(c, &t, &src, outcomes, was_random, check_invariants);
  tab_free(&t);
  return rc;
}

/* Output rows of one shot from its recorded outcomes: the outcomes
 * themselves (outputs 0), or each detector's XOR of its records followed by
 * each observable's (outputs 1). */
static int n_rows(const oracle_circuit* c, int outputs) { return outputs ? c->ndet + c->nobs : c->nmeas; }

static void shot_rows(const oracle_circuit* c, int outputs, const uint8_t* oc, uint8_t* rows) {
  if (!outputs) {
    memcpy(rows, oc, (size_t)c->nmeas);
    return;
  }
  memset(rows, 0, (size_t)(c->ndet + c->nobs));
  int d = 0;
  for (int i = 0; i < c->nops; i++) {
    const op_t* op = &c->ops[i];
    if (op->kind == OP_DET) {
      for (int j = 0; j < op->ntargets; j++) rows[d] ^= oc[op->targets[j]];
      d++;
    } else if (op->kind == OP_OBS) {
      for (int j = 1; j < op->ntargets; j++) rows[c->ndet + op->targets[0]] ^= oc[op->targets[j]];
    }
  }
}

int oracle_output_dims(const oracle_circuit* c, int* n_detectors, int* n_observables) {
  if (!c) return fail(-1, "null argument");
  if (n_detectors) *n_detectors = c->ndet;
  if (n_observables) *n_observables = c->nobs;
  return 0;
}

int oracle_rows_from_outcomes(const oracle_circuit* c, int outputs, const uint8_t* outcomes, uint8_t* rows) {
  if (!c || !outcomes || !rows) return fail(-1, "null argument");
  shot_rows(c, outputs, outcomes, rows);
  return 0;
}

/* ------------------------------------------------------------------ */
/* many shots                                                          */
/* ------------------------------------------------------------------ */

typedef struct {
  const oracle_circuit* c;
  int outputs;
  uint64_t seed, first_shot, shots;
  uint64_t* out;
  size_t ld;
  const uint64_t* shot_ids;
  uint8_t* outcomes;
  uint64_t lo, hi;  /* word range (packed) or shot-index range (list) */
  int rc;
} job_t;

static void* sample_words(void* arg) {
  job_t* j = arg;
  const oracle_circuit* c = j->c;
  tab_t t;
  tab_alloc(&t, c->nq);
  const int nr = n_rows(c, j->outputs);
  uint8_t* oc = malloc((size_t)(c->nmeas ? c->nmeas : 1));
  uint8_t* rows = malloc((size_t)(nr ? nr : 1));
  for (uint64_t w = j->lo; w < j->hi && j->rc == 0; w++) {
    for (int b = 0; b < 64; b++) {
      uint64_t i = w * 64 + (uint64_t)b;
      if (i >= j->shots) break;
      codesrc_t src = {NULL, j->seed, j->first_shot + i};
      if ((j->rc = run_shot(c, &t, &src, oc, NULL, 0)) != 0) break;
      shot_rows(c, j->outputs, oc, rows);
      for (int k = 0; k < nr; k++)
        if (rows[k]) j->out[(size_t)k * j->ld + w] |= (uint64_t)1 << b;
    }
  }
  free(rows);
  free(oc);
  tab_free(&t);
  return NULL;
}

static void* sample_list(void* arg) {
  job_t* j = arg;
  const oracle_circuit* c = j->c;
  tab_t t;
  tab_alloc(&t, c->nq);
  const int nr = n_rows(c, j->outputs);
  uint8_t* oc = malloc((size_t)(c->nmeas ? c->nmeas : 1));
  for (uint64_t i = j->lo; i < j->hi && j->rc == 0; i++) {
    codesrc_t src = {NULL, j->seed, j->shot_ids[i]};
    if ((j->rc = run_shot(c, &t, &src, oc, NULL, 0)) != 0) break;
    shot_rows(c, j->outputs, oc, j->outcomes + i * (size_t)nr);
  }
  free(oc);
  tab_free(&t);
  return NULL;
}

static int pick_threads(int n_threads, uint64_t work) {
  if (n_threads <= 0) {
    long nc = sysconf(_SC_NPROCESSORS_ONLN);
    n_threads = nc > 0 ? (int)nc : 1;
  }
  if ((uint64_t)n_threads > work) n_threads = (int)(work ? work : 1);
  return n_threads;
}

static int run_jobs(job_t* proto, uint64_t work, int n_threads, void* (*fn)(void*)) {
  int nt = pick_threads(n_threads, work);
  job_t* jobs = calloc((size_t)nt, sizeof(job_t));
  pthread_t* th = calloc((size_t)nt, sizeof(pthread_t));
  for (int i = 0; i < nt; i++) {
    jobs[i] = *proto;
    jobs[i].lo = work * (uint64_t)i / (uint64_t)nt;
    jobs[i].hi = work * (uint64_t)(i + 1) / (uint64_t)nt;
    jobs[i].rc = 0;
  }
  for (int i = 1; i < nt; i++) pthread_create(&th[i], NULL, fn, &jobs[i]);
  fn(&jobs[0]);
  for (int i = 1; i < nt; i++) pthread_join(th[i], NULL);
  int rc = 0;
  for (int i = 0; i < nt; i++)
    if (jobs[i].rc) rc = jobs[i].rc;
  free(jobs);
  free(th);
  return rc;
}

int oracle_sample_outputs(const oracle_circuit* c, int outputs, uint64_t seed, uint64_t first_shot, uint64_t shots,
                          uint64_t* out, size_t ld, int n_threads) {
  if (!c || (!out && shots)) return fail(-1, "null argument");
  if (outputs != 0 && outputs != 1) return fail(-1, "unknown outputs %d", outputs);
  uint64_t words = (shots + 63) / 64;
  if (ld < words) return fail(-1, "ld %zu < %llu words", ld, (unsigned long long)words);
  memset(out, 0, (size_t)n_rows(c, outputs) * ld * 8);
  if (!shots) return 0;
  job_t proto = {c, outputs, seed, first_shot, shots, out, ld, NULL, NULL, 0, 0, 0};
  return run_jobs(&proto, words, n_threads, sample_words);
}

int oracle_sample(const oracle_circuit* c, uint64_t seed, uint64_t first_shot, uint64_t shots,
                  uint64_t* out, size_t ld, int n_threads) {
  return oracle_sample_outputs(c, 0, seed, first_shot, shots, out, ld, n_threads);
}

int oracle_sample_shots_outputs(const oracle_circuit* c, int outputs, uint64_t seed, const uint64_t* shot_ids,
                                size_t n, uint8_t* rows, int n_threads) {
  if (!c || (n && (!shot_ids || !rows))) return fail(-1, "null argument");
  if (outputs != 0 && outputs != 1) return fail(-1, "unknown outputs %d", outputs);
  if (!n) return 0;
  job_t proto = {c, outputs, seed, 0, 0, NULL, 0, shot_ids, rows, 0, 0, 0};
  return run_jobs(&proto, n, n_threads, sample_list);
}

int oracle_sample_shots(const oracle_circuit* c, uint64_t seed, const uint64_t* shot_ids,
                        size_t n, uint8_t* outcomes, int n_threads) {
  return oracle_sample_shots_outputs(c, 0, seed, shot_ids, n, outcomes, n_threads);
}
