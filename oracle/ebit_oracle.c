/*
 * EBIT interface step: CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow, single-threaded FP64
 * reference that the GPU library is checked against. Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it. The product
 * library never links, loads or calls it, and the two share no source.
 *
 * It follows Pan, Long, Chirco, Scardovelli, Popinet and Zaleski, "An
 * Edge-based Interface Tracking (EBIT) Method for Multiphase-flow Simulation
 * with Surface Tension" (arXiv 2309.00338):
 *   Sec. 2.1, Eq. (Eq_marker_dis)  explicit Euler marker advection with a
 *                                  bilinear velocity, split by direction into
 *                                  aligned and unaligned markers;
 *   Sec. 2.2                       circle fit through the advected chain;
 *   Sec. 2.3                       Color Vertex update on corners and centres;
 *   Sec. 2.4                       topology change driven by the corner CVs;
 *   Sec. 2.5                       volume fraction from markers + CVs, and
 *                                  height-function curvature of that fraction.
 *
 * Organisation (deliberately global, unlike the tiled GPU gather): one sweep
 * advects every marker, flips every crossed node, lands every aligned marker,
 * builds the old segment table of every cell, then walks each new unaligned
 * edge's crossing segments and chains, then sets every centre CV. The y sweep
 * is the x sweep applied to the transposed grid.
 *
 * Index space: node (i,j) sits at the integer point (i,j); cell (i,j) is
 * [i,i+1]x[j,j+1]. H(i,j) joins nodes (i,j),(i+1,j) and its marker sits at
 * (i+hoff, j); V(i,j) joins (i,j),(i,j+1) with its marker at (i, j+voff).
 * u[j][i] is the x-face velocity at (i, j+1/2); v[j][i] the y-face velocity at
 * (i+1/2, j). All arrays are row-major with x fastest.
 *
 * Readings of points the paper leaves open are marked "reading:" below.
 *
 * Build with -ffp-contract=off: the expression orders written here are the
 * definition, and no multiply-add may be fused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_CFL 3
#define OR_ERR_DOMAIN 4
#define OR_ERR_NOMEM 6

#define TIE_EPS 1e-12

/* Counters, in this exact order (the Python wrapper names them). */
enum {
  S_MARKERS = 0,      /* markers present at the start of each sweep (summed) */
  S_ANNIHILATED,      /* aligned landers dropped by a1 (pairs and outer pairs) */
  S_THREE_LANDERS,    /* new aligned edges that received three landers */
  S_TIES,             /* near-degenerate decisions (within 1e-12) */
  S_FIT_FALLBACK,     /* new unaligned markers placed by the straight line */
  S_FIT_REJECT,       /* circle roots discarded for leaving their edge */
  S_PARITY_FALLBACK,  /* colour parity and crossing parity disagree */
  S_THREE_CROSSINGS,  /* new unaligned edges crossed by three segments */
  S_CV_SET,           /* centre CVs set by the aligned-marker rule */
  S_CV_CONFLICT,      /* left and right edges of a cell disagree */
  S_CV_UNRESOLVED,    /* 4-marker cell whose centre CV found no rule */
  S_WALL_VIOLATION,   /* non-zero wall-normal displacement of a wall marker */
  S_INVARIANT_FAIL,   /* lander parity differs from the corner colours */
  S_HF_FAIL,          /* interfacial cells where both HF orientations fail */
  S_INTERFACIAL,      /* cells with two or more markers (curvature pass) */
  S_GHF_FIT,          /* of the HF failures, cells given kappa by the marker parabola */
  S_COUNT
};

/* ------------------------------------------------------------------------- */
/* Optional log of where ties happen (a decision within 1e-12 of degenerate:   */
/* a landed or new offset at a node, a crossing endpoint on the line, two      */
/* equal crossing heights, a root on the chord). Each entry is four int32:     */
/* kind, sweep direction, and the edge in the sweep frame (a along the sweep,  */
/* b across it): kind 1 the aligned edge (a, b), kinds 2-5 the new unaligned   */
/* edge on line a, row b. The oracle is single-threaded; the log is a static. */
/* ------------------------------------------------------------------------- */
enum { TIE_LANDED = 1, TIE_ENDPOINT = 2, TIE_HEIGHTS = 3, TIE_ROOT_SIDE = 4, TIE_NEW_OFFSET = 5 };
static int32_t *g_tie_log = NULL;
static int64_t g_tie_cap = 0, g_tie_n = 0;
static int g_tie_dir = 0, g_tie_a = 0, g_tie_b = 0;

static void note_tie(int64_t *st, int kind, int a, int b) {
  st[S_TIES]++;
  if (g_tie_log && g_tie_n < g_tie_cap) {
    int32_t *e = g_tie_log + 4 * g_tie_n;
    e[0] = kind;
    e[1] = g_tie_dir;
    e[2] = a;
    e[3] = b;
  }
  g_tie_n++;
}

/* Start logging into buf (cap entries of four int32; NULL stops logging) and
 * clear the count. */
void or_tie_log(int32_t *buf, int64_t cap) {
  g_tie_log = buf;
  g_tie_cap = buf ? cap : 0;
  g_tie_n = 0;
}

/* Ties seen since or_tie_log (may exceed the capacity; only cap are kept). */
int64_t or_tie_count(void) { return g_tie_n; }

/* ------------------------------------------------------------------------- */
/* The sweep frame: "a" runs along the sweep, "b" across it. For the x sweep   */
/* (a,b) = (i,j); for the y sweep the arrays are transposed first.            */
/* ------------------------------------------------------------------------- */
typedef struct {
  int na, nb;
  const uint8_t *col; /* (nb+1) x (na+1) */
  const uint8_t *cen; /* nb x na */
  const double *al;   /* (nb+1) x na   aligned-edge offsets */
  const double *un;   /* nb x (na+1)   unaligned-edge offsets */
  const double *vel;  /* nb x (na+1)   face velocity along the sweep */
  double lam;         /* dt / h */
  int line;           /* place new unaligned markers by the straight line (EBIT-SL) */
} frame;

#define NODE(F, a, b) ((size_t)(b) * (size_t)((F)->na + 1) + (size_t)(a))
#define ALE(F, a, b) ((size_t)(b) * (size_t)(F)->na + (size_t)(a))
#define UNE(F, a, b) ((size_t)(b) * (size_t)((F)->na + 1) + (size_t)(a))
#define CELL(F, a, b) ((size_t)(b) * (size_t)(F)->na + (size_t)(a))

static double lerp(double a, double b, double t) { return a + t * (b - a); }

/* Face velocity with mirrored ghost rows across the walls (reading: the
 * paper's bilinear interpolation on the staggered lattice, ghosts copy the
 * nearest interior face). */
static double vel_at(const frame *F, int a, int r) {
  if (r < 0) r = 0;
  if (r > F->nb - 1) r = F->nb - 1;
  return F->vel[UNE(F, a, r)];
}

/* A marker reference: kind 0 = aligned edge (a,b), kind 1 = unaligned (a,b). */
typedef struct {
  int kind, a, b;
} mref;

/* Per-sweep scratch shared by the steps below. */
typedef struct {
  double *sp;      /* aligned: unnormalised advected offset s' */
  double *dv;      /* unaligned: displacement d along the sweep */
  uint8_t *ncol;   /* new node colours */
  int8_t *target;  /* aligned: landing shift -1/0/+1 */
  uint8_t *kept;   /* aligned: this lander is the one kept on its new edge */
  int8_t *seg;     /* old cell segments: 4 edge ids per cell, -1 when absent */
  /* per new unaligned edge: the fitted crossing's chain, for the centre CV */
  uint8_t *zhas;
  mref *zP1, *zP2, *zP3, *zP4;
  uint8_t *zhas1, *zhas4;
  int64_t *st;
  int err;
} sweep_ws;

static int present_al(const frame *F, const uint8_t *col, int a, int b) {
  return col[NODE(F, a, b)] != col[NODE(F, a + 1, b)];
}
static int present_un(const frame *F, const uint8_t *col, int a, int b) {
  return col[NODE(F, a, b)] != col[NODE(F, a, b + 1)];
}

/* Edge e of cell (p,q): 0 bottom, 1 right, 2 top, 3 left. */
static mref edge_marker(int p, int q, int e) {
  mref m;
  switch (e) {
    case 0: m.kind = 0; m.a = p; m.b = q; break;
    case 1: m.kind = 1; m.a = p + 1; m.b = q; break;
    case 2: m.kind = 0; m.a = p; m.b = q + 1; break;
    default: m.kind = 1; m.a = p; m.b = q; break;
  }
  return m;
}

/* Old segments of cell (p,q) (Sec. 2.3): two markers form one segment; four
 * markers form two, each joining the pair around a corner whose colour differs
 * from the centre CV ("isolated" corner). Corner k lies between edges k-1 and
 * k (k = 0 BL, 1 BR, 2 TR, 3 TL). Segments are listed by ascending corner. */
static void cell_segments(const frame *F, int p, int q, int8_t out[4]) {
  const uint8_t *c = F->col;
  int k[4];
  k[0] = c[NODE(F, p, q)];
  k[1] = c[NODE(F, p + 1, q)];
  k[2] = c[NODE(F, p + 1, q + 1)];
  k[3] = c[NODE(F, p, q + 1)];
  int pres[4];
  pres[0] = k[0] != k[1];
  pres[1] = k[1] != k[2];
  pres[2] = k[3] != k[2];
  pres[3] = k[0] != k[3];
  int n = pres[0] + pres[1] + pres[2] + pres[3];
  out[0] = out[1] = out[2] = out[3] = -1;
  if (n == 2) {
    int w = 0;
    for (int e = 0; e < 4; e++)
      if (pres[e]) out[w++] = (int8_t)e;
  } else if (n == 4) {
    int cc = F->cen[CELL(F, p, q)];
    int w = 0;
    for (int corner = 0; corner < 4; corner++) {
      if (k[corner] != cc) {
        out[w++] = (int8_t)((corner + 3) % 4);
        out[w++] = (int8_t)corner;
      }
    }
  }
}

/* Local coordinates of an advected marker relative to node (a0,b0). Aligned
 * markers move along their line (blue points); unaligned ones move off it by
 * d (gray points). */
static void adv_point(const frame *F, const sweep_ws *W, mref m, int a0, int b0, double *X, double *Y) {
  if (m.kind == 0) {
    *X = (double)(m.a - a0) + W->sp[ALE(F, m.a, m.b)];
    *Y = (double)(m.b - b0);
  } else {
    *X = (double)(m.a - a0) + W->dv[UNE(F, m.a, m.b)];
    *Y = (double)(m.b - b0) + F->un[UNE(F, m.a, m.b)];
  }
}

/* "Left of line a = a0" iff x < a0, evaluated exactly on the offset. */
static int left_of(const frame *F, const sweep_ws *W, mref m, int a0) {
  if (m.kind == 0) return W->sp[ALE(F, m.a, m.b)] < (double)(a0 - m.a);
  return W->dv[UNE(F, m.a, m.b)] < (double)(a0 - m.a);
}

/* Chain neighbour of the marker on edge e of old cell (p,q), away from that
 * cell: its partner in the cell across edge e. Returns 0 at a wall. */
static int chain_neighbour(const frame *F, const sweep_ws *W, int p, int q, int e, mref *out) {
  int pp = p, qq = q;
  switch (e) {
    case 0: qq = q - 1; break;
    case 1: pp = p + 1; break;
    case 2: qq = q + 1; break;
    default: pp = p - 1; break;
  }
  if (pp < 0 || pp >= F->na || qq < 0 || qq >= F->nb) return 0;
  int eo = (e + 2) % 4;
  const int8_t *s = W->seg + 4 * CELL(F, pp, qq);
  for (int k = 0; k < 4; k += 2) {
    if (s[k] < 0) continue;
    if (s[k] == eo) { *out = edge_marker(pp, qq, s[k + 1]); return 1; }
    if (s[k + 1] == eo) { *out = edge_marker(pp, qq, s[k]); return 1; }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Circle fit (Sec. 2.2).                                                      */
/* reading: points 1,2,3,4 are the advected chain P1-P2-P3-P4 around the        */
/* crossing segment P2P3, P2 on the left of the line. Circle A passes through  */
/* P1,P2,P3 and circle B through P2,P3,P4; each is used when its outer point    */
/* exists ("whenever it is possible"). Each circle is written as the           */
/* generalised circle a(X^2+Y^2) + bX + cY + e = 0 through three points; on     */
/* the line X = 0 it reduces to aY^2 + cY + e = 0.                              */
/* ------------------------------------------------------------------------- */

/* One circle's root on X = 0, or 0 when unavailable. (Xo,Yo) is the outer
 * point (P1 or P4); the kept root lies strictly across chord P2P3 from it,
 * i.e. on the arc P2 -> P3 that continues the curve. */
static int circle_root(double Xa, double Ya, double Xb, double Yb, double Xc, double Yc,
                       double Xo, double Yo, double X2, double Y2, double X3, double Y3,
                       double ysl, double *root, int64_t *st) {
  double Qa = Xa * Xa + Ya * Ya;
  double Qb = Xb * Xb + Yb * Yb;
  double Qc = Xc * Xc + Yc * Yc;
  /* coefficients of the determinant |X^2+Y^2 X Y 1; rows of the 3 points| */
  double ca = Xa * (Yb - Yc) + Xb * (Yc - Ya) + Xc * (Ya - Yb);
  double cc = Qa * (Xb - Xc) + Qb * (Xc - Xa) + Qc * (Xa - Xb);
  double ce = -(Qa * (Xb * Yc - Xc * Yb) + Qb * (Xc * Ya - Xa * Yc) + Qc * (Xa * Yb - Xb * Ya));
  double r;
  if (ca == 0.0) {
    if (cc == 0.0) return 0; /* degenerate: all three points coincide */
    r = -ce / cc;            /* collinear: the line through them */
  } else {
    double disc = cc * cc - 4.0 * ca * ce;
    if (disc < 0.0) disc = 0.0;
    double sq = sqrt(disc);
    double q = -0.5 * (cc + (cc >= 0.0 ? sq : -sq));
    double r1, r2;
    if (q == 0.0) {
      r1 = 0.0;
      r2 = 0.0;
    } else {
      r1 = q / ca;
      r2 = ce / q;
    }
    double DX = X3 - X2, DY = Y3 - Y2;
    double L2 = DX * DX + DY * DY;
    double so = DX * (Yo - Y2) - DY * (Xo - X2);
    double s1 = DX * (r1 - Y2) - DY * (0.0 - X2);
    double s2 = DX * (r2 - Y2) - DY * (0.0 - X2);
    if (fabs(s1) < TIE_EPS * L2 || fabs(s2) < TIE_EPS * L2) note_tie(st, TIE_ROOT_SIDE, g_tie_a, g_tie_b);
    int q1 = (s1 > 0.0 && so < 0.0) || (s1 < 0.0 && so > 0.0);
    int q2 = (s2 > 0.0 && so < 0.0) || (s2 < 0.0 && so > 0.0);
    if (q1 && !q2) r = r1;
    else if (q2 && !q1) r = r2;
    else r = (fabs(r1 - ysl) <= fabs(r2 - ysl)) ? r1 : r2;
  }
  if (!(r >= 0.0 && r <= 1.0)) { /* reading: a root off its edge is discarded */
    st[S_FIT_REJECT]++;
    return 0;
  }
  *root = r;
  return 1;
}

/* Straight-line intersection of chord P2P3 with X = 0 (the EBIT-SL value),
 * clamped to the edge. */
static double line_y(double X2, double Y2, double X3, double Y3) {
  double y = Y2 + (Y3 - Y2) * (0.0 - X2) / (X3 - X2);
  if (y < 0.0) y = 0.0;
  if (y > 1.0) y = 1.0;
  return y;
}

/* ------------------------------------------------------------------------- */
/* One sweep along "a" (Fig. EBIT_advection).                                  */
/* ------------------------------------------------------------------------- */
static int sweep_frame(const frame *F, uint8_t *ncol_out, uint8_t *ncen, double *nal, double *nun, int64_t *st) {
  const int na = F->na, nb = F->nb;
  const size_t n_nodes = (size_t)(na + 1) * (nb + 1);
  const size_t n_al = (size_t)na * (nb + 1);
  const size_t n_un = (size_t)(na + 1) * nb;
  const size_t n_cells = (size_t)na * nb;
  sweep_ws W;
  memset(&W, 0, sizeof W);
  W.st = st;
  W.sp = calloc(n_al, sizeof(double));
  W.dv = calloc(n_un, sizeof(double));
  W.ncol = ncol_out;
  W.target = calloc(n_al, 1);
  W.kept = calloc(n_al, 1);
  W.seg = malloc(4 * n_cells);
  W.zhas = calloc(n_un, 1);
  W.zhas1 = calloc(n_un, 1);
  W.zhas4 = calloc(n_un, 1);
  W.zP1 = calloc(n_un, sizeof(mref));
  W.zP2 = calloc(n_un, sizeof(mref));
  W.zP3 = calloc(n_un, sizeof(mref));
  W.zP4 = calloc(n_un, sizeof(mref));
  int rc = OR_OK;
  if (!W.sp || !W.dv || !W.target || !W.kept || !W.seg || !W.zhas || !W.zhas1 || !W.zhas4 || !W.zP1 ||
      !W.zP2 || !W.zP3 || !W.zP4) {
    rc = OR_ERR_NOMEM;
    goto done;
  }

  /* (1) Advect every marker by Eq. (Eq_marker_dis): X' = X + U dt, U bilinear. */
  for (int b = 0; b <= nb; b++)
    for (int a = 0; a < na; a++) {
      if (!present_al(F, F->col, a, b)) continue;
      st[S_MARKERS]++;
      double s = F->al[ALE(F, a, b)];
      double ub = lerp(lerp(vel_at(F, a, b - 1), vel_at(F, a + 1, b - 1), s),
                       lerp(vel_at(F, a, b), vel_at(F, a + 1, b), s), 0.5);
      double d = ub * F->lam;
      if (fabs(d) > 0.5) rc = OR_ERR_CFL;
      W.sp[ALE(F, a, b)] = s + d;
    }
  for (int b = 0; b < nb; b++)
    for (int a = 0; a <= na; a++) {
      if (!present_un(F, F->col, a, b)) continue;
      st[S_MARKERS]++;
      double t = F->un[UNE(F, a, b)];
      double ub = t < 0.5 ? lerp(vel_at(F, a, b - 1), vel_at(F, a, b), t + 0.5)
                          : lerp(vel_at(F, a, b), vel_at(F, a, b + 1), t - 0.5);
      double d = ub * F->lam;
      if (fabs(d) > 0.5) rc = OR_ERR_CFL;
      if (a == 0 || a == na) { /* reading: closed walls hold their markers */
        if (d != 0.0) st[S_WALL_VIOLATION]++;
        d = 0.0;
      }
      W.dv[UNE(F, a, b)] = d;
    }

  /* (2) Corner CVs: a node changes colour when a marker crosses it (Sec. 2.3). */
  memcpy(W.ncol, F->col, n_nodes);
  for (int b = 0; b <= nb; b++)
    for (int a = 0; a < na; a++) {
      if (!present_al(F, F->col, a, b)) continue;
      double sp = W.sp[ALE(F, a, b)];
      if (sp >= 1.0) {
        if (a + 1 >= na) { rc = OR_ERR_DOMAIN; continue; }
        W.target[ALE(F, a, b)] = 1;
        W.ncol[NODE(F, a + 1, b)] ^= 1;
      } else if (sp < 0.0) {
        if (a == 0) { rc = OR_ERR_DOMAIN; continue; }
        W.target[ALE(F, a, b)] = -1;
        W.ncol[NODE(F, a, b)] ^= 1;
      }
    }

  /* (3) Aligned landing and topology change (Sec. 2.4): one marker per edge;
   * an even number of landers annihilates; of three, the one that did not
   * change edge is kept (reading). */
  for (int b = 0; b <= nb; b++)
    for (int a = 0; a < na; a++) {
      int src[3], n = 0;
      if (a - 1 >= 0 && present_al(F, F->col, a - 1, b) && W.target[ALE(F, a - 1, b)] == 1) src[n++] = a - 1;
      if (present_al(F, F->col, a, b) && W.target[ALE(F, a, b)] == 0 && W.sp[ALE(F, a, b)] >= 0.0 &&
          W.sp[ALE(F, a, b)] < 1.0)
        src[n++] = a;
      if (a + 1 < na && present_al(F, F->col, a + 1, b) && W.target[ALE(F, a + 1, b)] == -1) src[n++] = a + 1;
      int keep = -1;
      if (n == 1) keep = src[0];
      if (n == 3) {
        keep = src[1];
        st[S_THREE_LANDERS]++;
      }
      st[S_ANNIHILATED] += n - (n & 1);
      int newpres = W.ncol[NODE(F, a, b)] != W.ncol[NODE(F, a + 1, b)];
      if (newpres != (n & 1)) st[S_INVARIANT_FAIL]++;
      if (keep >= 0) {
        W.kept[ALE(F, keep, b)] = 1;
        double sp = W.sp[ALE(F, keep, b)];
        double o = keep < a ? sp - 1.0 : (keep > a ? sp + 1.0 : sp);
        nal[ALE(F, a, b)] = o;
        if (o < TIE_EPS || 1.0 - o < TIE_EPS) note_tie(st, TIE_LANDED, a, b);
      }
    }

  /* (4) Old connectivity: the segments of every cell before the advection. */
  for (int q = 0; q < nb; q++)
    for (int p = 0; p < na; p++) cell_segments(F, p, q, W.seg + 4 * CELL(F, p, q));

  /* (5) New unaligned markers (red points): where the new corner CVs differ,
   * the advected segments crossing the line give the crossing; the circle fit
   * through the chain gives its position (Sec. 2.2). */
  memcpy(nun, F->un, n_un * sizeof(double)); /* wall lines keep their markers */
  for (int b = 0; b < nb; b++)
    for (int a = 1; a < na; a++) {
      if (W.ncol[NODE(F, a, b)] == W.ncol[NODE(F, a, b + 1)]) continue;
      /* crossing segments of old cells (a-1,b) then (a,b) */
      int cp[4], cl[4], cr[4], nx = 0;
      double X2v[4], Y2v[4], X3v[4], Y3v[4], ysl[4];
      for (int p = a - 1; p <= a; p++) {
        const int8_t *s = W.seg + 4 * CELL(F, p, b);
        for (int k = 0; k < 4; k += 2) {
          if (s[k] < 0) continue;
          mref m1 = edge_marker(p, b, s[k]), m2 = edge_marker(p, b, s[k + 1]);
          int l1 = left_of(F, &W, m1, a), l2 = left_of(F, &W, m2, a);
          if (l1 == l2) continue;
          cp[nx] = p;
          cl[nx] = l1 ? s[k] : s[k + 1];
          cr[nx] = l1 ? s[k + 1] : s[k];
          adv_point(F, &W, edge_marker(p, b, cl[nx]), a, b, &X2v[nx], &Y2v[nx]);
          adv_point(F, &W, edge_marker(p, b, cr[nx]), a, b, &X3v[nx], &Y3v[nx]);
          ysl[nx] = line_y(X2v[nx], Y2v[nx], X3v[nx], Y3v[nx]);
          nx++;
        }
      }
      int pick = -1;
      if (nx == 1) pick = 0;
      else if (nx == 3) {
        /* reading: an odd count above one takes the median crossing */
        st[S_THREE_CROSSINGS]++;
        for (int x = 0; x < 3 && pick < 0; x++) {
          int below = 0;
          for (int y = 0; y < 3; y++) {
            if (y == x) continue;
            if (ysl[y] < ysl[x] || (ysl[y] == ysl[x] && y < x)) below++;
          }
          if (below == 1) pick = x;
        }
        for (int x = 0; x < 3; x++)
          for (int y = x + 1; y < 3; y++)
            if (fabs(ysl[x] - ysl[y]) < TIE_EPS) note_tie(st, TIE_HEIGHTS, a, b);
      }
      if (pick < 0) { /* reading: colours decide presence; place mid-edge */
        st[S_PARITY_FALLBACK]++;
        nun[UNE(F, a, b)] = 0.5;
        continue;
      }
      double X2 = X2v[pick], Y2 = Y2v[pick], X3 = X3v[pick], Y3 = Y3v[pick];
      if (fabs(X2) < TIE_EPS || fabs(X3) < TIE_EPS) note_tie(st, TIE_ENDPOINT, a, b);
      g_tie_a = a; /* where a root-side tie inside the circle fit belongs */
      g_tie_b = b;
      int p = cp[pick];
      mref m2 = edge_marker(p, b, cl[pick]), m3 = edge_marker(p, b, cr[pick]), m1, m4;
      int h1 = chain_neighbour(F, &W, p, b, cl[pick], &m1);
      int h4 = chain_neighbour(F, &W, p, b, cr[pick], &m4);
      double y;
      if (X3 == 0.0) {
        y = Y3;
      } else if (F->line) {
        /* EBIT-SL, the method's first version (Sec. 2.2 and the SL rows of
         * Tables 1, 3, 4, 5): the new marker is where the straight segment
         * P2P3 crosses the grid line */
        y = ysl[pick];
      } else {
        double X1 = 0, Y1 = 0, X4 = 0, Y4 = 0, rA = 0, rB = 0;
        int okA = 0, okB = 0;
        if (h1) {
          adv_point(F, &W, m1, a, b, &X1, &Y1);
          okA = circle_root(X1, Y1, X2, Y2, X3, Y3, X1, Y1, X2, Y2, X3, Y3, ysl[pick], &rA, st);
        }
        if (h4) {
          adv_point(F, &W, m4, a, b, &X4, &Y4);
          okB = circle_root(X2, Y2, X3, Y3, X4, Y4, X4, Y4, X2, Y2, X3, Y3, ysl[pick], &rB, st);
        }
        if (okA && okB) y = (rA + rB) * 0.5;
        else if (okA) y = rA;
        else if (okB) y = rB;
        else {
          y = ysl[pick];
          st[S_FIT_FALLBACK]++;
        }
      }
      nun[UNE(F, a, b)] = y;
      if (y < TIE_EPS || 1.0 - y < TIE_EPS) note_tie(st, TIE_NEW_OFFSET, a, b);
      size_t z = UNE(F, a, b);
      W.zhas[z] = 1;
      W.zP1[z] = m1;
      W.zP2[z] = m2;
      W.zP3[z] = m3;
      W.zP4[z] = m4;
      W.zhas1[z] = (uint8_t)h1;
      W.zhas4[z] = (uint8_t)h4;
    }

  /* (6) Centre CVs (Sec. 2.3, rules (1)-(5)). reading: for the new unaligned
   * marker on the cell's left edge (then its right edge), the bracketing
   * endpoint on the cell's side is the first candidate and, if it is an
   * unaligned (gray) point, its chain neighbour the second. A candidate that
   * is an aligned marker kept on the cell's bottom or top edge isolates the
   * corner it shares with the new marker's edge; the centre takes the other
   * colour. Otherwise the centre keeps its value. */
  for (int b = 0; b < nb; b++)
    for (int a = 0; a < na; a++) {
      int res[2] = {-1, -1};
      for (int side = 0; side < 2; side++) {
        int line = a + side;
        if (line <= 0 || line >= na) continue;
        size_t z = UNE(F, line, b);
        if (!W.zhas[z]) continue;
        mref cand[2];
        int nc = 0;
        mref first = side == 0 ? W.zP3[z] : W.zP2[z];
        cand[nc++] = first;
        if (first.kind == 1) {
          if (side == 0 && W.zhas4[z]) cand[nc++] = W.zP4[z];
          if (side == 1 && W.zhas1[z]) cand[nc++] = W.zP1[z];
        }
        for (int k = 0; k < nc; k++) {
          mref m = cand[k];
          if (m.kind != 0) continue;
          size_t id = ALE(F, m.a, m.b);
          if (!W.kept[id]) continue;
          if (m.a + W.target[id] != a) continue;
          if (m.b != b && m.b != b + 1) continue;
          res[side] = 1 - W.ncol[NODE(F, line, m.b)];
          break;
        }
      }
      int cc = F->cen[CELL(F, a, b)];
      if (res[0] >= 0) {
        cc = res[0];
        st[S_CV_SET]++;
        if (res[1] >= 0 && res[1] != res[0]) st[S_CV_CONFLICT]++;
      } else if (res[1] >= 0) {
        cc = res[1];
        st[S_CV_SET]++;
      } else {
        const uint8_t *c = W.ncol;
        int k0 = c[NODE(F, a, b)], k1 = c[NODE(F, a + 1, b)], k2 = c[NODE(F, a + 1, b + 1)],
            k3 = c[NODE(F, a, b + 1)];
        if ((k0 != k1) + (k1 != k2) + (k3 != k2) + (k0 != k3) == 4) st[S_CV_UNRESOLVED]++;
      }
      ncen[CELL(F, a, b)] = (uint8_t)cc;
    }

done:
  free(W.sp);
  free(W.dv);
  free(W.target);
  free(W.kept);
  free(W.seg);
  free(W.zhas);
  free(W.zhas1);
  free(W.zhas4);
  free(W.zP1);
  free(W.zP2);
  free(W.zP3);
  free(W.zP4);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Public sweep/step entry points (state updated in place).                   */
/* ------------------------------------------------------------------------- */

static void transpose_u8(const uint8_t *src, uint8_t *dst, int rows, int cols) {
  for (int r = 0; r < rows; r++)
    for (int c = 0; c < cols; c++) dst[(size_t)c * rows + r] = src[(size_t)r * cols + c];
}
static void transpose_f64(const double *src, double *dst, int rows, int cols) {
  for (int r = 0; r < rows; r++)
    for (int c = 0; c < cols; c++) dst[(size_t)c * rows + r] = src[(size_t)r * cols + c];
}

/* dir 0: sweep along x with u; dir 1: along y with v. flags bit 1: EBIT-SL. */
int or_sweep(int nx, int ny, double h, uint8_t *c, uint8_t *cc, double *hoff, double *voff, const double *u,
             const double *v, double dt, int dir, int flags, int64_t *st) {
  if (nx < 4 || ny < 4 || !(h > 0.0)) return OR_ERR_ARG;
  const size_t n_nodes = (size_t)(nx + 1) * (ny + 1), n_cells = (size_t)nx * ny;
  const size_t n_h = (size_t)nx * (ny + 1), n_v = (size_t)(nx + 1) * ny;
  double lam = dt / h;
  int rc;
  g_tie_dir = dir;
  if (dir == 0) {
    frame F = {nx, ny, c, cc, hoff, voff, u, lam, (flags >> 1) & 1};
    uint8_t *nc = malloc(n_nodes), *ncc = malloc(n_cells);
    double *nh = calloc(n_h, sizeof(double)), *nv = calloc(n_v, sizeof(double));
    if (!nc || !ncc || !nh || !nv) { free(nc); free(ncc); free(nh); free(nv); return OR_ERR_NOMEM; }
    rc = sweep_frame(&F, nc, ncc, nh, nv, st);
    memcpy(c, nc, n_nodes);
    memcpy(cc, ncc, n_cells);
    memcpy(hoff, nh, n_h * sizeof(double));
    memcpy(voff, nv, n_v * sizeof(double));
    free(nc); free(ncc); free(nh); free(nv);
    return rc;
  }
  /* y sweep: transpose so that y runs along the frame's "a" axis. */
  uint8_t *tc = malloc(n_nodes), *tcc = malloc(n_cells), *nc = malloc(n_nodes), *ncc = malloc(n_cells);
  double *tal = malloc(n_v * sizeof(double)), *tun = malloc(n_h * sizeof(double));
  double *tvel = malloc(n_h * sizeof(double));
  double *nal = calloc(n_v, sizeof(double)), *nun = calloc(n_h, sizeof(double));
  if (!tc || !tcc || !nc || !ncc || !tal || !tun || !tvel || !nal || !nun) {
    rc = OR_ERR_NOMEM;
    goto out;
  }
  transpose_u8(c, tc, ny + 1, nx + 1);
  transpose_u8(cc, tcc, ny, nx);
  transpose_f64(voff, tal, ny, nx + 1); /* V edges are aligned with y */
  transpose_f64(hoff, tun, ny + 1, nx); /* H edges are unaligned */
  transpose_f64(v, tvel, ny + 1, nx);
  {
    frame F = {ny, nx, tc, tcc, tal, tun, tvel, lam, (flags >> 1) & 1};
    rc = sweep_frame(&F, nc, ncc, nal, nun, st);
  }
  transpose_u8(nc, c, nx + 1, ny + 1);
  transpose_u8(ncc, cc, nx, ny);
  transpose_f64(nal, voff, nx + 1, ny);
  transpose_f64(nun, hoff, nx, ny + 1);
out:
  free(tc); free(tcc); free(nc); free(ncc); free(tal); free(tun); free(tvel); free(nal); free(nun);
  return rc;
}

/* One time step = two sweeps (Sec. 2.1). reading: step n runs x then y when n
 * is even and y then x when n is odd, unless flags bit 0 (x then y always) is
 * set. flags bit 1: EBIT-SL placement of new unaligned markers. */
int or_step(int nx, int ny, double h, uint8_t *c, uint8_t *cc, double *hoff, double *voff, const double *u,
            const double *v, double dt, int64_t step, int flags, int64_t *st) {
  int first = ((flags & 1) || (step % 2) == 0) ? 0 : 1;
  int rc1 = or_sweep(nx, ny, h, c, cc, hoff, voff, u, v, dt, first, flags, st);
  int rc2 = or_sweep(nx, ny, h, c, cc, hoff, voff, u, v, dt, 1 - first, flags, st);
  return rc1 ? rc1 : rc2;
}

/* ------------------------------------------------------------------------- */
/* Volume fraction (Sec. 2.5): area of the colour-1 part of each cell, the     */
/* interface being the straight segment(s) between the cell's markers.        */
/* ------------------------------------------------------------------------- */
static double cell_fraction(int nx, int ny, const uint8_t *c, const uint8_t *cc, const double *hoff,
                            const double *voff, int i, int j, int *nmark) {
  size_t W1 = (size_t)nx + 1;
  int kBL = c[(size_t)j * W1 + i], kBR = c[(size_t)j * W1 + i + 1];
  int kTR = c[(size_t)(j + 1) * W1 + i + 1], kTL = c[(size_t)(j + 1) * W1 + i];
  int pb = kBL != kBR, pr = kBR != kTR, pt = kTL != kTR, pl = kBL != kTL;
  int n = pb + pr + pt + pl;
  *nmark = n;
  (void)ny;
  if (n == 0) return (double)kBL;
  double hb = pb ? hoff[(size_t)j * nx + i] : 0.0;
  double ht = pt ? hoff[(size_t)(j + 1) * nx + i] : 0.0;
  double vl = pl ? voff[(size_t)j * W1 + i] : 0.0;
  double vr = pr ? voff[(size_t)j * W1 + i + 1] : 0.0;
  if (n == 2) {
    /* shoelace over the colour-1 corners and the two markers, walking the
     * cell boundary counter-clockwise from the bottom-left corner */
    double px[6], py[6];
    int m = 0;
    if (kBL) { px[m] = 0.0; py[m] = 0.0; m++; }
    if (pb) { px[m] = hb; py[m] = 0.0; m++; }
    if (kBR) { px[m] = 1.0; py[m] = 0.0; m++; }
    if (pr) { px[m] = 1.0; py[m] = vr; m++; }
    if (kTR) { px[m] = 1.0; py[m] = 1.0; m++; }
    if (pt) { px[m] = ht; py[m] = 1.0; m++; }
    if (kTL) { px[m] = 0.0; py[m] = 1.0; m++; }
    if (pl) { px[m] = 0.0; py[m] = vl; m++; }
    double acc = 0.0;
    for (int k = 0; k < m; k++) {
      int k1 = (k + 1 == m) ? 0 : k + 1;
      acc += px[k] * py[k1] - px[k1] * py[k];
    }
    return 0.5 * acc;
  }
  /* four markers: the two isolated corner triangles carry their corner's
   * colour, the central hexagon carries the centre CV (Sec. 2.3) */
  int cen = cc[(size_t)j * nx + i];
  double tBL = 0.5 * (hb * vl), tBR = 0.5 * ((1.0 - hb) * vr);
  double tTR = 0.5 * ((1.0 - vr) * (1.0 - ht)), tTL = 0.5 * (ht * (1.0 - vl));
  double s = (kBL != cen) ? tBL + tTR : tBR + tTL;
  return cen ? 1.0 - s : s;
}

int or_fraction(int nx, int ny, const uint8_t *c, const uint8_t *cc, const double *hoff, const double *voff,
                double *C) {
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      int n;
      C[(size_t)j * nx + i] = cell_fraction(nx, ny, c, cc, hoff, voff, i, j, &n);
    }
  return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Height-function curvature of C (Sec. 2.5) on a fixed 7x3 stencil.          */
/* reading: orientation from the corner CVs (the CV distribution gives the     */
/* normal direction, Sec. 2.3), as exact integer sums; walls mirror cells and  */
/* nodes; kappa > 0 for a convex colour-1 region, in physical units.           */
/* ------------------------------------------------------------------------- */
static int mirror_cell(int k, int n) {
  if (k < 0) return -1 - k;
  if (k >= n) return 2 * n - 1 - k;
  return k;
}
static int mirror_node(int k, int n) {
  if (k < 0) return -k;
  if (k > n) return 2 * n - k;
  return k;
}

static int cell_markers(int nx, const uint8_t *c, int i, int j) {
  size_t W1 = (size_t)nx + 1;
  int kBL = c[(size_t)j * W1 + i], kBR = c[(size_t)j * W1 + i + 1];
  int kTR = c[(size_t)(j + 1) * W1 + i + 1], kTL = c[(size_t)(j + 1) * W1 + i];
  return (kBL != kBR) + (kBR != kTR) + (kTL != kTR) + (kBL != kTL);
}

/* Heights along columns (rows == 0) or rows (rows == 1) around cell (i,j).
 * Returns 1 and kappa on success. */
static int hf_try(int nx, int ny, double h, const uint8_t *c, const double *C, int i, int j, int rows, double *kap) {
  double y[3];
  int sig = 0;
  for (int k = -1; k <= 1; k++) {
    int ci = 0, cj = 0, ei0, ej0, ei1, ej1;
    if (!rows) {
      ci = mirror_cell(i + k, nx);
      ei0 = ci; ej0 = mirror_cell(j - 3, ny);
      ei1 = ci; ej1 = mirror_cell(j + 3, ny);
    } else {
      cj = mirror_cell(j + k, ny);
      ei0 = mirror_cell(i - 3, nx); ej0 = cj;
      ei1 = mirror_cell(i + 3, nx); ej1 = cj;
    }
    if (cell_markers(nx, c, ei0, ej0) != 0 || cell_markers(nx, c, ei1, ej1) != 0) return 0;
    int c0 = c[(size_t)ej0 * (nx + 1) + ei0], c1 = c[(size_t)ej1 * (nx + 1) + ei1];
    if (c0 == c1) return 0;
    int s = c0 == 1 ? 1 : -1; /* colour 1 at the low end of the stencil */
    if (sig == 0) sig = s;
    else if (sig != s) return 0;
    double S = 0.0;
    for (int m = -3; m <= 3; m++) {
      if (!rows) S += C[(size_t)mirror_cell(j + m, ny) * nx + ci];
      else S += C[(size_t)cj * nx + mirror_cell(i + m, nx)];
    }
    y[k + 1] = sig == 1 ? S - 3.0 : 4.0 - S;
  }
  double hx = (y[2] - y[0]) * 0.5;
  double hxx = y[2] - 2.0 * y[1] + y[0];
  double g = 1.0 + hx * hx;
  *kap = (-(double)sig * hxx) / (h * g * sqrt(g));
  return 1;
}

/* Fallback where no height is valid: Sec. 2.5 computes kappa by the
 * generalised height-function method, which fits a parabola to interface
 * points, in a frame aligned with the interface normal, when heights are
 * missing. reading: EBIT's markers are those points, and the normal is the
 * integer node-colour gradient (gx, gy) used for the HF orientation, pointing
 * into colour 1. All markers on the edges of the 5x5 cells around (i,j) that
 * lie inside the grid, relative to the cell centre in index units, are
 * projected on the tangent (X) and the normal (Y) and fitted by least squares
 * with Y = a + b X + c X^2 (normal equations solved by Cramer's rule); kappa =
 * 2c / (1 + b^2)^(3/2) / h, positive for convex colour 1. Fails with fewer
 * than three points, a zero gradient or a degenerate system. The points are
 * taken H edges first (rows y, then x), then V edges. */
/* The fit itself on n points (px, py), exported for its pins. */
int or_parabola_fit(int n, const double *px, const double *py, double xc, double yc, int gx, int gy, double h,
                    double *kap) {
  if (gx == 0 && gy == 0) return 0;
  const double gl = sqrt((double)gx * (double)gx + (double)gy * (double)gy);
  const double nX = (double)gx / gl, nY = (double)gy / gl; /* unit normal into colour 1 */
  double S0 = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0, T0 = 0.0, T1 = 0.0, T2 = 0.0;
  for (int k = 0; k < n; k++) {
    const double dx = px[k] - xc, dy = py[k] - yc;
    const double X = dx * (-nY) + dy * nX; /* along the tangent */
    const double Y = dx * nX + dy * nY;    /* along the normal */
    const double X2 = X * X;
    S0 += 1.0;
    S1 += X;
    S2 += X2;
    S3 += X2 * X;
    S4 += X2 * X2;
    T0 += Y;
    T1 += X * Y;
    T2 += X2 * Y;
  }
  if (S0 < 3.0) return 0;
  const double det = S0 * (S2 * S4 - S3 * S3) - S1 * (S1 * S4 - S3 * S2) + S2 * (S1 * S3 - S2 * S2);
  if (!(det > 1e-10 * (S0 * S2 * S4))) return 0;
  const double db = S0 * (T1 * S4 - S3 * T2) - T0 * (S1 * S4 - S3 * S2) + S2 * (S1 * T2 - T1 * S2);
  const double dc = S0 * (S2 * T2 - T1 * S3) - S1 * (S1 * T2 - T1 * S2) + T0 * (S1 * S3 - S2 * S2);
  const double b = db / det, cc = dc / det;
  const double g = 1.0 + b * b;
  *kap = (2.0 * cc) / (h * g * sqrt(g));
  return 1;
}

static int ghf_fit(int nx, int ny, double h, const uint8_t *c, const double *hoff, const double *voff, int i, int j,
                   int gx, int gy, double *kap) {
  const size_t W1 = (size_t)nx + 1;
  double px[66], py[66];
  int n = 0;
  for (int pass = 0; pass < 2; pass++)
    for (int y = j - 2; y <= j + 2 + (pass == 0); y++)
      for (int x = i - 2; x <= i + 2 + (pass == 1); x++) {
        if (pass == 0) { /* H(x,y) */
          if (x < 0 || x >= nx || y < 0 || y > ny) continue;
          if (c[(size_t)y * W1 + x] == c[(size_t)y * W1 + x + 1]) continue;
          px[n] = x + hoff[(size_t)y * nx + x];
          py[n] = y;
        } else { /* V(x,y) */
          if (x < 0 || x > nx || y < 0 || y >= ny) continue;
          if (c[(size_t)y * W1 + x] == c[(size_t)(y + 1) * W1 + x]) continue;
          px[n] = x;
          py[n] = y + voff[(size_t)y * W1 + x];
        }
        n++;
      }
  return or_parabola_fit(n, px, py, i + 0.5, j + 0.5, gx, gy, h, kap);
}

int or_curvature(int nx, int ny, double h, const uint8_t *c, const double *hoff, const double *voff, const double *C,
                 double *K, int64_t *st) {
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t id = (size_t)j * nx + i;
      if (cell_markers(nx, c, i, j) < 2) {
        K[id] = 0.0;
        continue;
      }
      st[S_INTERFACIAL]++;
      int ncx = 0, ncy = 0;
      for (int m = j - 1; m <= j + 2; m++) {
        size_t r = (size_t)mirror_node(m, ny) * (nx + 1);
        ncx += c[r + mirror_node(i + 2, nx)] + c[r + mirror_node(i + 1, nx)] - c[r + mirror_node(i, nx)] -
               c[r + mirror_node(i - 1, nx)];
      }
      for (int l = i - 1; l <= i + 2; l++) {
        size_t col = (size_t)mirror_node(l, nx);
        ncy += c[(size_t)mirror_node(j + 2, ny) * (nx + 1) + col] + c[(size_t)mirror_node(j + 1, ny) * (nx + 1) + col] -
               c[(size_t)mirror_node(j, ny) * (nx + 1) + col] - c[(size_t)mirror_node(j - 1, ny) * (nx + 1) + col];
      }
      int first_rows = abs(ncy) >= abs(ncx) ? 0 : 1;
      double kap;
      if (hf_try(nx, ny, h, c, C, i, j, first_rows, &kap) || hf_try(nx, ny, h, c, C, i, j, 1 - first_rows, &kap)) {
        K[id] = kap;
      } else {
        st[S_HF_FAIL]++;
        /* the node sums point into colour 1 */
        if (ghf_fit(nx, ny, h, c, hoff, voff, i, j, ncx, ncy, &kap)) {
          K[id] = kap;
          st[S_GHF_FIT]++;
        } else {
          K[id] = NAN;
        }
      }
    }
  return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Consumers of the interface on the same grid (Sec. 2.5, Eq. physical and    */
/* the surface-tension term of Eq. NS).                                        */
/* ------------------------------------------------------------------------- */
/* Eq. (physical) with the Heaviside function approximated by C:
 * rho = C rho1 + (1 - C) rho2 and mu = C mu1 + (1 - C) mu2 in every cell.
 * Surface tension as a continuum face force sigma kappa_f grad C (the delta
 * function times the normal approximated by the gradient of C across the
 * face): on the x-face between cells (i-1,j) and (i,j),
 *   fx = sigma * kf * (C(i,j) - C(i-1,j)) / h,
 * reading: kf is the curvature of the face's two cells that carry it (two or
 * more markers and a finite value), their mean when both do, else 0; wall
 * faces carry no force. fy likewise on the y-faces. Any output may be NULL. */
static int curv_defined(int nx, const uint8_t *c, const double *K, int i, int j) {
  return cell_markers(nx, c, i, j) >= 2 && isfinite(K[(size_t)j * nx + i]);
}

static double face_kappa(int nx, const uint8_t *c, const double *K, int ia, int ja, int ib, int jb) {
  int da = curv_defined(nx, c, K, ia, ja), db = curv_defined(nx, c, K, ib, jb);
  double ka = K[(size_t)ja * nx + ia], kb = K[(size_t)jb * nx + ib];
  if (da && db) return (ka + kb) * 0.5;
  if (da) return ka;
  if (db) return kb;
  return 0.0;
}

int or_ns_fields(int nx, int ny, double h, const uint8_t *c, const double *C, const double *K, double rho1,
                 double rho2, double mu1, double mu2, double sigma, double *rho, double *mu, double *fx, double *fy) {
  if (nx < 4 || ny < 4 || !(h > 0.0)) return OR_ERR_ARG;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      size_t id = (size_t)j * nx + i;
      if (rho) rho[id] = C[id] * rho1 + (1.0 - C[id]) * rho2;
      if (mu) mu[id] = C[id] * mu1 + (1.0 - C[id]) * mu2;
    }
  if (fx)
    for (int j = 0; j < ny; j++)
      for (int i = 0; i <= nx; i++) {
        double f = 0.0;
        if (i > 0 && i < nx) {
          double cl = C[(size_t)j * nx + i - 1], cr = C[(size_t)j * nx + i];
          if (cl != cr) f = sigma * face_kappa(nx, c, K, i - 1, j, i, j) * (cr - cl) / h;
        }
        fx[(size_t)j * (nx + 1) + i] = f;
      }
  if (fy)
    for (int j = 0; j <= ny; j++)
      for (int i = 0; i < nx; i++) {
        double f = 0.0;
        if (j > 0 && j < ny) {
          double cb = C[(size_t)(j - 1) * nx + i], ct = C[(size_t)j * nx + i];
          if (cb != ct) f = sigma * face_kappa(nx, c, K, i, j - 1, i, j) * (ct - cb) / h;
        }
        fy[(size_t)j * nx + i] = f;
      }
  return OR_OK;
}

int or_counter_count(void) { return S_COUNT; }
