// CTMRG expectation values (ntu_ctm_*; declared in include/ntu.h).  The host
// code here only orders device work: every contraction is a permutation of
// axes and a complex product on the GPU (k_ctm.hip), in the same steps as the
// environment of a two-site checkerboard is built by directional moves.
//
// Lattice: A on (x, y) with x + y even, B on the others; the r leg of (x, y)
// joins the l leg of (x + 1, y), the t leg joins the b leg of (x, y + 1).
// Environment of each position of the 2 x 2 cell: corners C1 (top left, legs
// r, b), C2 (top right, l, b), C3 (bottom right, t, l), C4 (bottom left, t, r)
// and edges T1 (top: l, r, b), T2 (right: t, b, l), T3 (bottom: l, r, t), T4
// (left: t, b, r); the inner legs of the edges carry the double-layer bond.
// One iteration is four left moves, the lattice turned a quarter turn
// clockwise after each.  A left move absorbs column x (x = 0, then 1) into the
// left environment of column x + 1; the fused legs on each cut between two
// rows go through the isometry Z of that cut: the chi leading left singular
// vectors of rho = H_u H_d^T, the half-system density matrix of the 2 x 2
// block around the cut.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>
#include "ntu.h"
#include "ctm.h"
#include "kernels.h"

#define NTU_CTM_CHECK(x) do { ntu_status s_ = (x); if (s_) return s_; } while (0)

namespace {


struct Tn {
  cd* p = nullptr;
  int r = 0;
  int s[ntu::CTM_MAX_RANK] = {};
  long long n() const {
    long long k = 1;
    for (int i = 0; i < r; ++i) k *= s[i];
    return k;
  }
};

Tn shaped(cd* p, std::initializer_list<int> sh) {
  Tn t;
  t.p = p;
  for (int v : sh) t.s[t.r++] = v;
  return t;
}

struct EnvT {
  Tn C[4], T[4];  // C1..C4, T1..T4
};

}  // namespace

struct ntu_ctm {
  int device = 0, p = 2, D = 2, chi = 4;
  hipStream_t stream = nullptr;
  std::string err;
  // persistent: a pool of uniform buffers for the environment and the site
  // double layers; the arena for the temporaries of one move or evaluation
  cd* pool = nullptr;
  long long slot_el = 0;
  int nslot = 0;
  std::vector<int> free_slots;
  cd* arena = nullptr;
  long long arena_el = 0, arena_top = 0;
  unsigned long long* norm_slot = nullptr;
  cd* scalars = nullptr;  // 256 values of an evaluation (network values)
  cd* gemm_ws = nullptr;  // partial sums of split products (CTM_GEMM_WS entries)
  EnvT env[2][2];
  int env_slot[2][2][8];
  Tn site[2][2];
  int site_slot[2][2];
  bool have_env = false;
};

namespace {

ntu_status cfail(ntu_ctm* c, ntu_status s, const std::string& m) {
  if (c) c->err = m;
  else ntu::set_global_error(m.c_str());
  return s;
}

// ---------------------------------------------------------------- memory
cd* arena_get(ntu_ctm* c, long long n) {
  const long long a = (n + 31) & ~31ll;
  if (c->arena_top + a > c->arena_el) return nullptr;
  cd* p = c->arena + c->arena_top;
  c->arena_top += a;
  return p;
}
int slot_get(ntu_ctm* c) {
  if (c->free_slots.empty()) return -1;
  int s = c->free_slots.back();
  c->free_slots.pop_back();
  return s;
}
void slot_put(ntu_ctm* c, int s) {
  if (s >= 0) c->free_slots.push_back(s);
}
cd* slot_ptr(ntu_ctm* c, int s) { return c->pool + (long long)s * c->slot_el; }

// ---------------------------------------------------------------- einsum
struct Err {
  hipError_t e = hipSuccess;
  std::string what;
  void set(hipError_t x, const char* w) {
    if (e == hipSuccess && x != hipSuccess) {
      e = x;
      what = w;
    }
  }
};

Tn alloc(ntu_ctm* c, Err& E, const int* sh, int r) {
  Tn t;
  t.r = r;
  for (int i = 0; i < r; ++i) t.s[i] = sh[i];
  t.p = arena_get(c, t.n());
  if (!t.p) E.set(hipErrorOutOfMemory, "ctm arena");
  return t;
}

Tn permute(ntu_ctm* c, Err& E, const Tn& x, const int* perm, bool conj) {
  bool id = !conj;
  for (int i = 0; i < x.r && id; ++i) id = perm[i] == i;
  if (id) return x;
  int sh[ntu::CTM_MAX_RANK];
  for (int i = 0; i < x.r; ++i) sh[i] = x.s[perm[i]];
  Tn y = alloc(c, E, sh, x.r);
  if (E.e != hipSuccess) return y;
  E.set(ntu::ctm_permute(x.p, y.p, x.r, x.s, perm, conj, c->stream), "permute");
  return y;
}

Tn reshape(const Tn& x, std::initializer_list<int> sh) {
  Tn y;
  y.p = x.p;
  for (int v : sh) y.s[y.r++] = v;
  return y;
}

// out = contraction of A and B over the labels they share and the output
// lacks ("ab,bc->ac"); every label appears in two of the three parts.
Tn contract(ntu_ctm* c, Err& E, const char* spec, const Tn& A, bool cA, const Tn& B, bool cB) {
  Tn none;
  if (E.e != hipSuccess) return none;
  const char* comma = std::strchr(spec, ',');
  const char* arrow = std::strstr(spec, "->");
  const std::string la(spec, comma), lb(comma + 1, arrow), lo(arrow + 2);
  if ((int)la.size() != A.r || (int)lb.size() != B.r) {
    E.set(hipErrorInvalidValue, "contract: rank");
    return none;
  }
  auto dim_of = [&](char ch) -> int {
    size_t i = la.find(ch);
    if (i != std::string::npos) return A.s[i];
    return B.s[lb.find(ch)];
  };
  std::string freeA, freeB, sum;
  for (char ch : la) (lo.find(ch) != std::string::npos ? freeA : sum) += ch;
  for (char ch : lb)
    if (lo.find(ch) != std::string::npos) freeB += ch;
  for (char ch : sum)
    if (lb.find(ch) == std::string::npos || A.s[la.find(ch)] != B.s[lb.find(ch)]) {
      E.set(hipErrorInvalidValue, "contract: label");
      return none;
    }
  for (char ch : lb)
    if (lo.find(ch) == std::string::npos && la.find(ch) == std::string::npos) {
      E.set(hipErrorInvalidValue, "contract: label");
      return none;
    }
  long long M = 1, N = 1, K = 1;
  for (char ch : freeA) M *= dim_of(ch);
  for (char ch : freeB) N *= dim_of(ch);
  for (char ch : sum) K *= dim_of(ch);
  if (K > 0 && K < 1024 && M * K <= 65536 && K * N <= 65536 && M * N <= 65536) {
    // small: one launch gathers the operands from their own layouts and
    // writes the result in the output's order (no permuted copies)
    int sh[ntu::CTM_MAX_RANK], r = 0;
    for (char ch : lo) sh[r++] = dim_of(ch);
    Tn C = alloc(c, E, sh, r);
    if (E.e != hipSuccess) return none;
    auto strides = [](const int* s, int rk, long long* st) {
      long long v = 1;
      for (int i = rk - 1; i >= 0; --i) {
        st[i] = v;
        v *= s[i];
      }
    };
    long long sa[ntu::CTM_MAX_RANK], sb[ntu::CTM_MAX_RANK], so[ntu::CTM_MAX_RANK];
    strides(A.s, A.r, sa);
    strides(B.s, B.r, sb);
    strides(sh, r, so);
    auto axes = [&](const std::string& labels, const std::string& in, const long long* st) {
      ntu::CtmAxes g;
      for (char ch : labels) {
        g.dim[g.n] = dim_of(ch);
        g.stride[g.n++] = st[in.find(ch)];
      }
      return g;
    };
    ntu::CtmGather gd;
    gd.ra = axes(freeA, la, sa);
    gd.ca = axes(sum, la, sa);
    gd.rb = axes(sum, lb, sb);
    gd.cb = axes(freeB, lb, sb);
    gd.rc = axes(freeA, lo, so);
    gd.cc = axes(freeB, lo, so);
    gd.conj_a = cA;
    gd.conj_b = cB;
    E.set(ntu::ctm_gemm_gather(A.p, B.p, C.p, (int)M, (int)N, (int)K, gd, c->stream), "gemm");
    if (lo.empty()) C.r = 0;
    return C;
  }
  int pa[ntu::CTM_MAX_RANK], pb[ntu::CTM_MAX_RANK], k = 0;
  for (char ch : freeA) pa[k++] = (int)la.find(ch);
  for (char ch : sum) pa[k++] = (int)la.find(ch);
  k = 0;
  for (char ch : sum) pb[k++] = (int)lb.find(ch);
  for (char ch : freeB) pb[k++] = (int)lb.find(ch);
  const Tn Ap = permute(c, E, A, pa, cA);
  const Tn Bp = permute(c, E, B, pb, cB);
  int sh[ntu::CTM_MAX_RANK], r = 0;
  const std::string mid = freeA + freeB;
  for (char ch : mid) sh[r++] = dim_of(ch);
  Tn C = alloc(c, E, sh, r);
  if (E.e != hipSuccess) return none;
  if (K == 0 || M * N == 0) E.set(ntu::ctm_zero(C.p, M * N, c->stream), "zero");
  else E.set(ntu::ctm_gemm(Ap.p, Bp.p, C.p, (int)M, (int)N, (int)K, c->gemm_ws, ntu::CTM_GEMM_WS, c->stream), "gemm");
  if (mid == lo || lo.empty()) {
    if (lo.empty()) C.r = 0;
    return C;
  }
  int po[ntu::CTM_MAX_RANK];
  for (int i = 0; i < (int)lo.size(); ++i) po[i] = (int)mid.find(lo[i]);
  return permute(c, E, C, po, false);
}

// every launch below is skipped once an error is recorded: a failed step
// leaves empty tensors (no data) behind it
void normalise(ntu_ctm* c, Err& E, Tn& t) {
  if (E.e != hipSuccess || !t.p) return;
  E.set(ntu::ctm_normalise(t.p, t.n(), c->norm_slot, c->stream), "norm");
}

// copy a temporary into a pool slot
Tn keep(ntu_ctm* c, Err& E, const Tn& t, int* slot) {
  Tn k = t;
  if (E.e != hipSuccess) return k;
  const int s = slot_get(c);
  if (s < 0 || t.n() > c->slot_el) {
    E.set(hipErrorOutOfMemory, "ctm pool");
    return k;
  }
  k.p = slot_ptr(c, s);
  E.set(hipMemcpyAsync(k.p, t.p, t.n() * sizeof(cd), hipMemcpyDeviceToDevice, c->stream), "copy");
  *slot = s;
  return k;
}

// ---------------------------------------------------------------- double layer
// a[(t t'), (l l'), (b b'), (r r')] = sum conj(T[s', t', ...]) O[s', s] T[s, t, ...]
Tn double_layer(ntu_ctm* c, Err& E, const Tn& T, const Tn* O) {
  const int D = c->D;
  Tn OT = O ? contract(c, E, "xs,stlbr->xtlbr", *O, false, T, false) : T;
  Tn a = contract(c, E, "xtlbr,xTLBR->tTlLbBrR", T, true, OT, false);
  return reshape(a, {D * D, D * D, D * D, D * D});
}

// ---------------------------------------------------------------- moves
Tn cut_density(ntu_ctm* c, Err& E, int x, int y) {
  const int x1 = (x + 1) % 2, y1 = (y + 1) % 2;
  const EnvT &tl = c->env[x][y1], &tr = c->env[x1][y1], &br = c->env[x1][y], &bl = c->env[x][y];
  const Tn &atl = c->site[x][y1], &atr = c->site[x1][y1], &abr = c->site[x1][y], &abl = c->site[x][y];
  // enlarged corners (see the file comment for the legs)
  Tn t = contract(c, E, "ab,aRu->bRu", tl.C[0], false, tl.T[0], false);
  t = contract(c, E, "bRu,bBl->RuBl", t, false, tl.T[3], false);
  Tn q1 = contract(c, E, "RuBl,uldr->RrBd", t, false, atl, false);
  t = contract(c, E, "ab,Lau->bLu", tr.C[1], false, tr.T[0], false);
  t = contract(c, E, "bLu,bBr->LuBr", t, false, tr.T[1], false);
  Tn q2 = contract(c, E, "LuBr,uldr->LlBd", t, false, atr, false);
  t = contract(c, E, "ab,Tar->bTr", br.C[2], false, br.T[1], false);
  t = contract(c, E, "bTr,Lbd->TrLd", t, false, br.T[2], false);
  Tn q3 = contract(c, E, "TrLd,uldr->TuLl", t, false, abr, false);
  t = contract(c, E, "ab,Tal->bTl", bl.C[3], false, bl.T[3], false);
  t = contract(c, E, "bTl,bRd->TlRd", t, false, bl.T[2], false);
  Tn q4 = contract(c, E, "TlRd,uldr->TuRr", t, false, abl, false);
  if (E.e != hipSuccess) return Tn();
  Tn Q1 = reshape(q1, {q1.s[0] * q1.s[1], q1.s[2] * q1.s[3]});
  Tn Q2 = reshape(q2, {q2.s[0] * q2.s[1], q2.s[2] * q2.s[3]});
  Tn Q3 = reshape(q3, {q3.s[0] * q3.s[1], q3.s[2] * q3.s[3]});
  Tn Q4 = reshape(q4, {q4.s[0] * q4.s[1], q4.s[2] * q4.s[3]});
  Tn Hu = contract(c, E, "ki,kw->iw", Q1, false, Q2, false);
  Tn Hd = contract(c, E, "jk,wk->jw", Q4, false, Q3, false);
  return contract(c, E, "iw,jw->ij", Hu, false, Hd, false);
}

// The isometries of the two cuts of column x (between rows y and y + 1, for
// y = 0, 1): one launch over both when their sizes agree.
void cut_isometries(ntu_ctm* c, Err& E, int x, Tn Z[2]) {
  Tn rho[2];
  for (int y = 0; y < 2; ++y) rho[y] = cut_density(c, E, x, y);
  if (E.e != hipSuccess) return;
  cd* ws[2] = {nullptr, nullptr};
  for (int y = 0; y < 2; ++y) {
    const int n = rho[y].s[0], k = n < c->chi ? n : c->chi;
    int zs[2] = {n, k};
    Z[y] = alloc(c, E, zs, 2);
    if (n > ntu::CTM_SVD_REG_NMAX) {
      ws[y] = arena_get(c, (long long)n * n + ntu::CTM_SVD_WS_EXTRA);
      if (!ws[y]) E.set(hipErrorOutOfMemory, "ctm arena");
    }
  }
  if (E.e != hipSuccess) return;
  if (rho[0].s[0] == rho[1].s[0]) {
    const cd* r2[2] = {rho[0].p, rho[1].p};
    cd* z2[2] = {Z[0].p, Z[1].p};
    E.set(ntu::ctm_svd_left(2, r2, rho[0].s[0], Z[0].s[1], z2, ws, c->stream), "svd");
  } else {
    for (int y = 0; y < 2 && E.e == hipSuccess; ++y)
      E.set(ntu::ctm_svd_left(1, &rho[y].p, rho[y].s[0], Z[y].s[1], &Z[y].p, &ws[y], c->stream), "svd");
  }
}

void left_move(ntu_ctm* c, Err& E) {
  for (int x = 0; x < 2 && E.e == hipSuccess; ++x) {
    const int x1 = (x + 1) % 2;
    c->arena_top = 0;
    Tn Z[2];
    cut_isometries(c, E, x, Z);
    Tn nC1[2], nT4[2], nC4[2];
    for (int y = 0; y < 2 && E.e == hipSuccess; ++y) {
      const EnvT& e = c->env[x][y];
      const Tn& a = c->site[x][y];
      const Tn &zu = Z[y], &zd = Z[(y + 1) % 2];
      // C1 of (x + 1, y): C1 T1, the down legs through Z of the cut above
      Tn t = contract(c, E, "ab,aRu->Rbu", e.C[0], false, e.T[0], false);
      t = reshape(t, {t.s[0], t.s[1] * t.s[2]});
      nC1[y] = contract(c, E, "Rn,nk->Rk", t, false, zu, true);
      // T4 of (x + 1, y): T4 a, up legs through Z above, down legs through Z below
      t = contract(c, E, "TBl,uldr->TuBdr", e.T[3], false, a, false);
      t = reshape(t, {t.s[0] * t.s[1], t.s[2] * t.s[3], t.s[4]});
      t = contract(c, E, "ik,ijr->kjr", zu, false, t, false);
      nT4[y] = contract(c, E, "kjr,jm->kmr", t, false, zd, true);
      // C4 of (x + 1, y): C4 T3, up legs through Z below
      t = contract(c, E, "ab,bRd->adR", e.C[3], false, e.T[2], false);
      t = reshape(t, {t.s[0] * t.s[1], t.s[2]});
      nC4[y] = contract(c, E, "ik,iR->kR", zd, false, t, false);
      normalise(c, E, nC1[y]);
      normalise(c, E, nT4[y]);
      normalise(c, E, nC4[y]);
    }
    for (int y = 0; y < 2 && E.e == hipSuccess; ++y) {
      EnvT& e = c->env[x1][y];
      int* sl = c->env_slot[x1][y];
      slot_put(c, sl[0]);
      slot_put(c, sl[7]);
      slot_put(c, sl[3]);
      e.C[0] = keep(c, E, nC1[y], &sl[0]);
      e.T[3] = keep(c, E, nT4[y], &sl[7]);
      e.C[3] = keep(c, E, nC4[y], &sl[3]);
    }
  }
}

// the lattice and its environment a quarter turn clockwise: (x, y) -> (y, -x)
void rotate(ntu_ctm* c, Err& E) {
  c->arena_top = 0;
  EnvT ne[2][2];
  int ns[2][2][8];
  Tn nsite[2][2];
  int nss[2][2];
  const int tr2[2] = {1, 0}, tr3[3] = {1, 0, 2}, rs[4] = {1, 2, 3, 0};
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int qx = y % 2, qy = (2 - x) % 2;
      const EnvT& e = c->env[x][y];
      const int* sl = c->env_slot[x][y];
      EnvT& o = ne[qx][qy];
      int* os = ns[qx][qy];
      // moved as they are
      o.C[0] = e.C[3]; os[0] = sl[3];
      o.C[2] = e.C[1]; os[2] = sl[1];
      o.T[1] = e.T[0]; os[5] = sl[4];
      o.T[3] = e.T[2]; os[7] = sl[6];
      // transposed into new slots
      o.C[1] = keep(c, E, permute(c, E, e.C[0], tr2, false), &os[1]);
      o.C[3] = keep(c, E, permute(c, E, e.C[2], tr2, false), &os[3]);
      o.T[0] = keep(c, E, permute(c, E, e.T[3], tr3, false), &os[4]);
      o.T[2] = keep(c, E, permute(c, E, e.T[1], tr3, false), &os[6]);
      slot_put(c, sl[0]);
      slot_put(c, sl[2]);
      slot_put(c, sl[7]);
      slot_put(c, sl[5]);
      nsite[qx][qy] = keep(c, E, permute(c, E, c->site[x][y], rs, false), &nss[qx][qy]);
      slot_put(c, c->site_slot[x][y]);
      c->arena_top = 0;
    }
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      c->env[x][y] = ne[x][y];
      std::memcpy(c->env_slot[x][y], ns[x][y], sizeof(ns[x][y]));
      c->site[x][y] = nsite[x][y];
      c->site_slot[x][y] = nss[x][y];
    }
}

void release_all(ntu_ctm* c) {
  c->free_slots.clear();
  for (int s = c->nslot - 1; s >= 0; --s) c->free_slots.push_back(s);
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      for (int k = 0; k < 8; ++k) c->env_slot[x][y][k] = -1;
      c->site_slot[x][y] = -1;
    }
}

// sites from A, B (widened to complex128 when real) and the identity boundary
void init_state(ntu_ctm* c, Err& E, const ntu_tensor* A, const ntu_tensor* B, bool reset) {
  const int D = c->D, p = c->p;
  const long long ns = (long long)p * D * D * D * D;
  c->arena_top = 0;
  Tn S[2];
  const ntu_tensor* in[2] = {A, B};
  for (int k = 0; k < 2; ++k) {
    S[k].p = arena_get(c, ns);
    S[k].r = 5;
    S[k].s[0] = p;
    for (int i = 1; i < 5; ++i) S[k].s[i] = D;
    if (!S[k].p) {
      E.set(hipErrorOutOfMemory, "ctm arena");
      return;
    }
    if (in[k]->dtype == NTU_F64) E.set(ntu::ctm_widen((const double*)in[k]->data, S[k].p, ns, c->stream), "widen");
    else E.set(hipMemcpyAsync(S[k].p, in[k]->data, ns * sizeof(cd), hipMemcpyDeviceToDevice, c->stream), "copy");
  }
  if (reset || !c->have_env) {
    release_all(c);
    // identity boundary: bond dimension 1, inner legs vec(1_D)
    std::vector<cd> e(D * D, cd{0.0, 0.0}), one(1, cd{1.0, 0.0});
    for (int i = 0; i < D; ++i) e[i * D + i] = cd{1.0, 0.0};
    for (int x = 0; x < 2; ++x)
      for (int y = 0; y < 2; ++y) {
        EnvT& en = c->env[x][y];
        int* sl = c->env_slot[x][y];
        for (int k = 0; k < 4 && E.e == hipSuccess; ++k) {
          sl[k] = slot_get(c);
          sl[4 + k] = slot_get(c);
          if (sl[k] < 0 || sl[4 + k] < 0) {
            E.set(hipErrorOutOfMemory, "ctm pool");
            break;
          }
          en.C[k] = shaped(slot_ptr(c, sl[k]), {1, 1});
          E.set(hipMemcpyAsync(en.C[k].p, one.data(), sizeof(cd), hipMemcpyHostToDevice, c->stream), "init");
          en.T[k] = shaped(slot_ptr(c, sl[4 + k]), {1, 1, D * D});
          E.set(hipMemcpyAsync(en.T[k].p, e.data(), sizeof(cd) * D * D, hipMemcpyHostToDevice, c->stream), "init");
        }
      }
    // the host vectors above must outlive the copies
    E.set(hipStreamSynchronize(c->stream), "init");
    c->have_env = true;
  } else {
    for (int x = 0; x < 2; ++x)
      for (int y = 0; y < 2; ++y) slot_put(c, c->site_slot[x][y]);
  }
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      Tn a = double_layer(c, E, S[(x + y) % 2], nullptr);
      c->site[x][y] = keep(c, E, a, &c->site_slot[x][y]);
    }
}

// ---------------------------------------------------------------- networks
Tn site_value(ntu_ctm* c, Err& E, const EnvT& e, const Tn& a) {
  // top row, then the left edge, the site, the right edge and the bottom row
  // (largest intermediate chi^2 D^4)
  Tn t = contract(c, E, "ab,aRu->bRu", e.C[0], false, e.T[0], false);
  Tn top = contract(c, E, "bRu,Rc->bcu", t, false, e.C[1], false);
  t = contract(c, E, "ab,bRd->aRd", e.C[3], false, e.T[2], false);
  Tn bot = contract(c, E, "aRd,cR->acd", t, false, e.C[2], false);
  t = contract(c, E, "bcu,bBl->cuBl", top, false, e.T[3], false);
  t = contract(c, E, "cuBl,uldr->cBdr", t, false, a, false);
  t = contract(c, E, "cBdr,cCr->BdC", t, false, e.T[1], false);
  return contract(c, E, "BdC,BCd->", t, false, bot, false);
}

Tn hbond_value(ntu_ctm* c, Err& E, const EnvT& eL, const EnvT& eR, const Tn& aL, const Tn& aR) {
  // largest intermediate chi^2 D^6
  Tn t = contract(c, E, "ab,aRu->bRu", eL.C[0], false, eL.T[0], false);
  t = contract(c, E, "bRu,RSv->buSv", t, false, eR.T[0], false);
  Tn top = contract(c, E, "buSv,Sc->bcuv", t, false, eR.C[1], false);
  t = contract(c, E, "ab,bRd->aRd", eL.C[3], false, eL.T[2], false);
  t = contract(c, E, "aRd,RSe->adSe", t, false, eR.T[2], false);
  Tn bot = contract(c, E, "adSe,cS->acde", t, false, eR.C[2], false);
  t = contract(c, E, "bcuv,bBl->cuvBl", top, false, eL.T[3], false);
  t = contract(c, E, "cuvBl,uldm->cvBdm", t, false, aL, false);
  t = contract(c, E, "cvBdm,vmen->cBden", t, false, aR, false);
  t = contract(c, E, "cBden,cCn->BdeC", t, false, eR.T[1], false);
  return contract(c, E, "BdeC,BCde->", t, false, bot, false);
}

ntu_status check_arg(ntu_ctm* c, const ntu_tensor* t, const char* name, std::initializer_list<long long> shape,
                     bool allow_real) {
  const std::string nm(name);
  if (!t || !t->data) return cfail(c, NTU_ERR_ARG, nm + ": NULL");
  if (!(t->dtype == NTU_C128 || (allow_real && t->dtype == NTU_F64)))
    return cfail(c, NTU_ERR_DTYPE, nm + ": element type");
  if (t->ndim != (int)shape.size()) return cfail(c, NTU_ERR_SHAPE, nm + ": rank");
  int i = 0;
  for (long long v : shape) {
    if (t->shape[i] != v) return cfail(c, NTU_ERR_SHAPE, nm + ": extent " + std::to_string(i));
    ++i;
  }
  long long st = 1;
  for (int k = t->ndim - 1; k >= 0; --k) {
    if (t->shape[k] != 1 && t->stride[k] != st) return cfail(c, NTU_ERR_SHAPE, nm + ": not dense row-major");
    st *= t->shape[k];
  }
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, t->data) != hipSuccess) {
    (void)hipGetLastError();
    return cfail(c, NTU_ERR_ARG, nm + ": not device memory");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return cfail(c, NTU_ERR_ARG, nm + ": not device memory");
  return NTU_OK;
}

struct Dev {
  int old = -1;
  explicit Dev(int d) {
    if (hipGetDevice(&old) == hipSuccess && old != d) (void)hipSetDevice(d);
    else old = -1;
  }
  ~Dev() {
    if (old >= 0) (void)hipSetDevice(old);
  }
};

}  // namespace

extern "C" {

ntu_status ntu_ctm_create(ntu_ctm** out, int device, int p, int D, int chi) {
  if (!out) return cfail(nullptr, NTU_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (p < 1 || p > 16 || D < 1 || D > 8 || chi < 1) return cfail(nullptr, NTU_ERR_SHAPE, "p in [1,16], D in [1,8], chi >= 1");
  if ((long long)chi * D * D > ntu::CTM_SVD_NMAX)
    return cfail(nullptr, NTU_ERR_SHAPE, "chi D^2 above " + std::to_string(ntu::CTM_SVD_NMAX));
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return cfail(nullptr, NTU_ERR_ARG, "no such device");
  Dev g(device);
  ntu_ctm* c = new ntu_ctm();
  c->device = device;
  c->p = p;
  c->D = D;
  c->chi = chi;
  const long long D2 = (long long)D * D, N = chi * D2;
  // pool: 32 environment tensors and 4 site double layers live, plus as many
  // in flight during a rotation
  c->slot_el = std::max<long long>({(long long)chi * chi * D2, D2 * D2 * D2 * D2, 64});
  c->nslot = 96;
  // arena: the temporaries of a column of a move (the cut matrices and
  // corners of both cuts, the isometries and SVD scratch, the absorbed edges:
  // terms of chi^2 D^6 and chi^2 D^4) or of an evaluation; the sum below
  // covers the peak of the allocation sequence with a third to spare for
  // D = 1..8 and chi D^2 up to 1024
  const long long cc = (long long)chi * chi;
  c->arena_el = std::max<long long>(1 << 20, 10 * cc * D2 * D2 * D2 + 64 * cc * D2 * D2 + 2 * N * N +
                                                 2 * ntu::CTM_SVD_WS_EXTRA + 8 * D2 * D2 * D2 * D2 + 8 * (long long)p * D2 * D2);
  hipError_t e = hipMalloc((void**)&c->pool, sizeof(cd) * c->slot_el * c->nslot);
  if (e == hipSuccess) e = hipMalloc((void**)&c->arena, sizeof(cd) * c->arena_el);
  if (e == hipSuccess) e = hipMalloc((void**)&c->norm_slot, 256);
  if (e == hipSuccess) e = hipMalloc((void**)&c->scalars, sizeof(cd) * 256);
  if (e == hipSuccess) e = hipMalloc((void**)&c->gemm_ws, sizeof(cd) * ntu::CTM_GEMM_WS);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(c->pool);
    (void)hipFree(c->arena);
    (void)hipFree(c->norm_slot);
    (void)hipFree(c->scalars);
    (void)hipFree(c->gemm_ws);
    delete c;
    return cfail(nullptr, NTU_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  release_all(c);
  *out = c;
  return NTU_OK;
}

ntu_status ntu_ctm_destroy(ntu_ctm* c) {
  if (!c) return NTU_OK;
  Dev g(c->device);
  (void)hipFree(c->pool);
  (void)hipFree(c->arena);
  (void)hipFree(c->norm_slot);
  (void)hipFree(c->scalars);
  (void)hipFree(c->gemm_ws);
  delete c;
  return NTU_OK;
}

ntu_status ntu_ctm_set_stream(ntu_ctm* c, void* stream) {
  if (!c) return cfail(nullptr, NTU_ERR_ARG, "ctm is NULL");
  c->stream = (hipStream_t)stream;
  return NTU_OK;
}

const char* ntu_ctm_last_error(const ntu_ctm* c) { return c ? c->err.c_str() : ""; }

ntu_status ntu_ctm_run(ntu_ctm* c, const ntu_tensor* A, const ntu_tensor* B, int n_iter, int reset) {
  if (!c) return cfail(nullptr, NTU_ERR_ARG, "ctm is NULL");
  if (n_iter < 0) return cfail(c, NTU_ERR_ARG, "n_iter must be >= 0");
  const long long p = c->p, D = c->D;
  NTU_CTM_CHECK(check_arg(c, A, "A", {p, D, D, D, D}, true));
  NTU_CTM_CHECK(check_arg(c, B, "B", {p, D, D, D, D}, true));
  Dev g(c->device);
  Err E;
  init_state(c, E, A, B, reset != 0);
  for (int it = 0; it < n_iter && E.e == hipSuccess; ++it)
    for (int m = 0; m < 4 && E.e == hipSuccess; ++m) {
      left_move(c, E);
      if (E.e == hipSuccess) rotate(c, E);
    }
  if (E.e != hipSuccess) {
    c->have_env = false;  // a move may be half done: the next run starts afresh
    return cfail(c, NTU_ERR_HIP, "ctm_run (" + E.what + "): " + hipGetErrorString(E.e));
  }
  return NTU_OK;
}

ntu_status ntu_ctm_expect(ntu_ctm* c, const ntu_tensor* A, const ntu_tensor* B, const ntu_tensor* ops1,
                          const ntu_tensor* ops2, ntu_tensor* out) {
  if (!c) return cfail(nullptr, NTU_ERR_ARG, "ctm is NULL");
  if (!c->have_env) return cfail(c, NTU_ERR_ARG, "no environment: call ntu_ctm_run first");
  const long long p = c->p, D = c->D;
  NTU_CTM_CHECK(check_arg(c, A, "A", {p, D, D, D, D}, true));
  NTU_CTM_CHECK(check_arg(c, B, "B", {p, D, D, D, D}, true));
  if (!ops1 || !ops2) return cfail(c, NTU_ERR_ARG, "ops: NULL");
  const long long n1 = ops1->ndim == 3 ? ops1->shape[0] : -1, n2 = ops2->ndim == 4 ? ops2->shape[0] : -1;
  if (n1 < 0 || n1 > 16 || n2 < 1 || n2 > 16)
    return cfail(c, NTU_ERR_SHAPE, "ops1: (n1 <= 16, p, p), ops2: (1..16, 2, p, p)");
  NTU_CTM_CHECK(check_arg(c, ops1, "ops1", {n1, p, p}, false));
  NTU_CTM_CHECK(check_arg(c, ops2, "ops2", {n2, 2, p, p}, false));
  NTU_CTM_CHECK(check_arg(c, out, "out", {2 * n1 + 4}, false));
  Dev g(c->device);
  Err E;
  const long long ns = p * D * D * D * D;
  // the site tensors (complex128) and their quarter-turned forms in pool slots
  const int rs[5] = {0, 2, 3, 4, 1};
  Tn S[2], SR[2];
  int sslot[4] = {-1, -1, -1, -1};
  const ntu_tensor* in[2] = {A, B};
  for (int k = 0; k < 2 && E.e == hipSuccess; ++k) {
    c->arena_top = 0;
    Tn t = shaped(arena_get(c, ns), {(int)p, (int)D, (int)D, (int)D, (int)D});
    if (!t.p) return cfail(c, NTU_ERR_HIP, "ctm arena");
    if (in[k]->dtype == NTU_F64) E.set(ntu::ctm_widen((const double*)in[k]->data, t.p, ns, c->stream), "widen");
    else E.set(hipMemcpyAsync(t.p, in[k]->data, ns * sizeof(cd), hipMemcpyDeviceToDevice, c->stream), "copy");
    S[k] = keep(c, E, t, &sslot[k]);
    SR[k] = keep(c, E, permute(c, E, t, rs, false), &sslot[2 + k]);
  }
  // scalars: one-site numerators and norms, then per bond the norm and the
  // values of the product terms
  cd* num1 = c->scalars;
  cd* den1 = num1 + 32;
  cd* den2 = den1 + 32;
  cd* term = den2 + 4;
  auto put = [&](const Tn& v, cd* dst) {
    if (E.e != hipSuccess || !v.p) return;
    E.set(hipMemcpyAsync(dst, v.p, sizeof(cd), hipMemcpyDeviceToDevice, c->stream), "copy");
  };
  const cd* o1 = (const cd*)ops1->data;
  const cd* o2 = (const cd*)ops2->data;
  auto op = [&](const cd* base) { return shaped(const_cast<cd*>(base), {(int)p, (int)p}); };
  // one-site values at (0, 0) (A) and (1, 0) (B)
  for (int s = 0; s < 2 && E.e == hipSuccess; ++s) {
    c->arena_top = 0;
    const EnvT& e = c->env[s][0];
    const Tn a = double_layer(c, E, S[s], nullptr);
    const Tn d = site_value(c, E, e, a);
    for (int k = 0; k < n1; ++k) put(d, den1 + 2 * k + s);
    for (int k = 0; k < n1 && E.e == hipSuccess; ++k) {
      const Tn Ok = op(o1 + (long long)k * p * p);
      const Tn aO = double_layer(c, E, S[s], &Ok);
      put(site_value(c, E, e, aO), num1 + 2 * k + s);
    }
  }
  // bonds H1 (0,0)-(1,0): A B; H2 (1,0)-(0,0): B A; the vertical bonds in the
  // lattice turned a quarter turn clockwise, with the site tensors turned:
  // V1 A(0,0)-B(0,1) -> (0,0)-(1,0), V2 B(0,1)-A(0,0) -> (1,0)-(0,0)
  for (int b = 0; b < 4 && E.e == hipSuccess; ++b) {
    const bool vert = b >= 2;
    if (b == 2) rotate(c, E);
    const int xl = b % 2, sl = b % 2, sr = 1 - sl;
    const Tn& TL = vert ? SR[sl] : S[sl];
    const Tn& TR = vert ? SR[sr] : S[sr];
    const EnvT &eL = c->env[xl][0], &eR = c->env[(xl + 1) % 2][0];
    c->arena_top = 0;
    const Tn aL = double_layer(c, E, TL, nullptr), aR = double_layer(c, E, TR, nullptr);
    put(hbond_value(c, E, eL, eR, aL, aR), den2 + b);
    for (int t = 0; t < n2 && E.e == hipSuccess; ++t) {
      c->arena_top = 0;
      const Tn O1 = op(o2 + (long long)t * 2 * p * p), O2 = op(o2 + (long long)t * 2 * p * p + p * p);
      const Tn bL = double_layer(c, E, TL, &O1), bR = double_layer(c, E, TR, &O2);
      put(hbond_value(c, E, eL, eR, bL, bR), term + b * n2 + t);
    }
  }
  // back to the original orientation
  rotate(c, E);
  rotate(c, E);
  rotate(c, E);
  cd* o = (cd*)out->data;
  if (E.e == hipSuccess) E.set(ntu::ctm_ratio(num1, den1, o, (int)(2 * n1), c->stream), "ratio");
  if (E.e == hipSuccess) E.set(ntu::ctm_sum_ratio(term, den2, o + 2 * n1, 4, (int)n2, c->stream), "ratio");
  for (int k = 0; k < 4; ++k) slot_put(c, sslot[k]);
  if (E.e != hipSuccess) {
    c->have_env = false;  // the turns may be half done: the next run starts afresh
    return cfail(c, NTU_ERR_HIP, "ctm_expect (" + E.what + "): " + hipGetErrorString(E.e));
  }
  return NTU_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Evolution run with CTMRG measurements (ntu_evolve)
// ---------------------------------------------------------------------------
hipStream_t ntu_internal_ctx_stream(const ntu_ctx* c);

namespace {

// item 0 of a batched (1, ...) descriptor as an unbatched one
ntu_tensor drop_batch(const ntu_tensor& t) {
  ntu_tensor r = t;
  r.ndim = t.ndim - 1;
  for (int i = 0; i + 1 < t.ndim; ++i) {
    r.shape[i] = t.shape[i + 1];
    r.stride[i] = t.stride[i + 1];
  }
  return r;
}

}  // namespace

extern "C" ntu_status ntu_evolve(ntu_ctx* ctx, ntu_ctm* c, ntu_tensor* A, ntu_tensor* B,
                                 const ntu_tensor* gate_factors, const ntu_step_opts* step,
                                 const ntu_evolve_opts* ev, const ntu_tensor* ops1, const ntu_tensor* hb,
                                 ntu_tensor* history, double* energy, int* n_meas, int* steps_done) {
  if (!c) return cfail(nullptr, NTU_ERR_ARG, "ctm is NULL");
  if (!ctx || !A || !B || !gate_factors || !step || !ev || !ops1 || !hb || !history || !n_meas || !steps_done)
    return cfail(c, NTU_ERR_ARG, "ntu_evolve: NULL argument");
  *n_meas = 0;
  *steps_done = 0;
  if (ev->n_steps < 0 || ev->measure_every < 1 || ev->ctm_iters < 1)
    return cfail(c, NTU_ERR_ARG, "ntu_evolve: n_steps >= 0, measure_every >= 1, ctm_iters >= 1");
  if (A->dtype == NTU_C64 || B->dtype == NTU_C64)
    return cfail(c, NTU_ERR_UNSUPPORTED, "ntu_evolve: complex64 storage (CTMRG takes complex128 or real tensors)");
  if (A->ndim != 6 || B->ndim != 6 || A->shape[0] != 1 || B->shape[0] != 1)
    return cfail(c, NTU_ERR_SHAPE, "ntu_evolve: A, B must be (1, p, D, D, D, D)");
  if (ops1->ndim != 3) return cfail(c, NTU_ERR_SHAPE, "ntu_evolve: ops1 must be (n1, p, p)");
  const long long width = 2 * ops1->shape[0] + 4;
  const long long need = ev->n_steps / ev->measure_every + 1;
  if (history->dtype != NTU_C128) return cfail(c, NTU_ERR_DTYPE, "ntu_evolve: history must be NTU_C128");
  if (history->ndim != 2 || history->shape[1] != width || history->shape[0] < need || history->stride[1] != 1 ||
      history->stride[0] != width || !history->data)
    return cfail(c, NTU_ERR_SHAPE, "ntu_evolve: history must be dense (max_meas >= " + std::to_string(need) +
                                       ", " + std::to_string(width) + ")");
  const ntu_tensor A0 = drop_batch(*A), B0 = drop_batch(*B);
  NTU_CTM_CHECK(check_arg(c, &A0, "A[0]", {c->p, c->D, c->D, c->D, c->D}, true));
  NTU_CTM_CHECK(check_arg(c, &B0, "B[0]", {c->p, c->D, c->D, c->D, c->D}, true));
  const hipStream_t st = ntu_internal_ctx_stream(ctx);
  const hipStream_t saved = c->stream;
  c->stream = st;
  int m = 0;
  auto measure = [&](bool reset, double& e) -> ntu_status {
    NTU_CTM_CHECK(ntu_ctm_run(c, &A0, &B0, ev->ctm_iters, reset ? 1 : 0));
    ntu_tensor row = *history;
    row.ndim = 1;
    row.shape[0] = width;
    row.stride[0] = 1;
    row.data = (cd*)history->data + (long long)m * width;
    NTU_CTM_CHECK(ntu_ctm_expect(c, &A0, &B0, ops1, hb, &row));
    cd v[4];
    Dev g(c->device);
    hipError_t he = hipMemcpyAsync(v, (cd*)row.data + (width - 4), sizeof v, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return cfail(c, NTU_ERR_HIP, std::string("ntu_evolve: ") + hipGetErrorString(he));
    e = 0.5 * (v[0].x + v[1].x + v[2].x + v[3].x);
    if (energy) energy[m] = e;
    *n_meas = ++m;
    return NTU_OK;
  };
  double e0 = 0.0;
  ntu_status s = measure(true, e0);
  for (int k = 1; s == NTU_OK && k <= ev->n_steps; ++k) {
    s = ntu_trotter_step(ctx, 1, A, B, gate_factors, step, nullptr);
    if (s != NTU_OK) break;
    *steps_done = k;
    if (k % ev->measure_every == 0) {
      double e = 0.0;
      s = measure(!ev->ctm_continue, e);
      if (s == NTU_OK && ev->energy_tol > 0.0 && std::fabs(e - e0) > ev->energy_tol) break;
    }
  }
  c->stream = saved;
  return s;
}
