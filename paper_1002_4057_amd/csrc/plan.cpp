// Host-side planner: task stream of the tile SPD inverse, hazard DAG,
// critical paths and the device dispatch order.  See plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <cstring>
#include <queue>
#include <unordered_map>
#include <utility>

namespace spdinv {
namespace {

struct Builder {
  const PlanOptions& o;
  int t, T;
  Plan* p;
  // hazard state over the paper's tile names (A, B, C copies)
  std::vector<int32_t> last_writer;
  std::vector<std::vector<int32_t>> readers;
  // predecessor lists, in program order
  std::vector<std::vector<int32_t>> preds;
  int cur_step = 0;
  int barrier = -1;  // barrier task that the current step's sources must follow

  // per tile row: the row has the renaming copy B (of L) / C (of L^{-1})
  bool rb(int i) const { return o.renamed && (o.ren_b.empty() || o.ren_b[i]); }
  bool rc(int i) const { return o.renamed && (o.ren_c.empty() || o.ren_c[i]); }

  // partial-sum tiles of the tree reduction: tile (i, j), segment l >= 1
  int zper = 0, zname = 0, zbase = 0;
  int Zh(int i, int j, int l) const { return zname + tri(i, j) * zper + (l - 1); }
  int Zd(int i, int j, int l) const { return zbase + tri(i, j) * zper + (l - 1); }

  Builder(const PlanOptions& opt, Plan* plan) : o(opt), t(opt.t), p(plan) {
    T = t * (t + 1) / 2;
    boff.assign(t, -1);
    coff.assign(t, -1);
    if (opt.steps != 7) {
      // the standard layout for the partial plans: the prologue of the
      // steps from a given factor writes B and D into it, and the solve's
      // right-hand sides follow D^T at 3T + 2t
      for (int i = 0; i < t; ++i) {
        boff[i] = T + tri(i, 0);
        coff[i] = 2 * T + tri(i, 0);
      }
      dbase = 3 * T;
    } else {
      // the inverse: the renamed rows of B, then those of C, then D (full
      // renaming: B at [T, 2T), C at [2T, 3T), D at 3T; in place: D at T)
      int next = T;
      for (int i = 0; i < t; ++i)
        if (rb(i)) {
          boff[i] = next;
          next += i + 1;
        }
      for (int i = 0; i < t; ++i)
        if (rc(i)) {
          coff[i] = next;
          next += i + 1;
        }
      dbase = next;
    }
    p->d_base = dbase;
    const int levels = std::min(std::max(opt.tree_levels, 0), 2);
    zper = (levels > 0 && (opt.steps & 2)) ? (1 << levels) - 1 : 0;
    zbase = dbase + 2 * t + t * opt.rhs_tiles;
    p->pool_tiles = (int64_t)zbase + (int64_t)T * zper;
    zname = 3 * T + t * opt.rhs_tiles;
    const size_t names = (size_t)zname + (size_t)T * zper;
    last_writer.assign(names, -1);
    readers.resize(names);
  }

  int tri(int i, int j) const { return i * (i + 1) / 2 + j; }
  // hazard names of the paper's tiles (A, and the copies B and C)
  int A(int i, int j) const { return tri(i, j); }
  int B(int i, int j) const { return T + tri(i, j); }
  int C(int i, int j) const { return 2 * T + tri(i, j); }
  // pool tiles of the copies (only renamed rows are stored) and of D, D^T
  std::vector<int> boff, coff;
  int dbase = 0;
  int Bd(int i, int j) const { return boff[i] + j; }
  int Cd(int i, int j) const { return coff[i] + j; }
  int D(int j) const { return dbase + j; }
  // right-hand-side tile (i, c): hazard name and pool index
  int Rh(int i, int c) const { return 3 * T + i + t * c; }
  int Rp(int i, int c) const { return dbase + 2 * t + i + t * c; }

  // Emits one task.  reads/writes are hazard names (A/B/C tile ids); the
  // device operands are given separately.
  int emit(int kind, int i, int j, int k, std::initializer_list<int> reads,
           std::initializer_list<int> writes, int out, int a, int b, int copy, int aux,
           int flags = 0) {
    const int v = (int)p->tasks.size();
    DevTask d;
    d.kind = kind | (flags << 8);
    d.out = out;
    d.a = a;
    d.b = b;
    d.copy = copy;
    d.aux = aux;
    d.succ_begin = d.succ_end = 0;
    p->tasks.push_back(d);
    p->step.push_back(cur_step);
    p->idx.push_back(((i & 1023) << 20) | ((j & 1023) << 10) | (k & 1023));
    std::vector<int32_t> pr;
    for (int r : reads)
      if (last_writer[r] >= 0) pr.push_back(last_writer[r]);  // RAW
    for (int w : writes) {
      if (last_writer[w] >= 0) pr.push_back(last_writer[w]);  // WAW
      for (int rd : readers[w]) pr.push_back(rd);             // WAR
    }
    std::sort(pr.begin(), pr.end());
    pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
    if (barrier >= 0) {
      bool has_same_step = false;
      for (int q : pr)
        if (p->step[q] == cur_step) { has_same_step = true; break; }
      if (!has_same_step) pr.push_back(barrier);
    }
    preds.push_back(std::move(pr));
    for (int r : reads) readers[r].push_back(v);
    for (int w : writes) {
      last_writer[w] = v;
      readers[w].clear();
    }
    return v;
  }

  // Barrier after the step just emitted: depends on that step's sinks.
  void emit_barrier() {
    const int v = (int)p->tasks.size();
    std::vector<char> has_succ(v, 0);
    for (int q = 0; q < v; ++q)
      for (int pr : preds[q]) has_succ[pr] = 1;
    std::vector<int32_t> pr;
    for (int q = 0; q < v; ++q)
      if (p->step[q] == cur_step && !has_succ[q]) pr.push_back(q);
    DevTask d{K_NOP, -1, -1, -1, -1, -1, 0, 0};
    p->tasks.push_back(d);
    p->step.push_back(0);
    p->idx.push_back(0);
    preds.push_back(std::move(pr));
    barrier = v;
  }

  int Dt(int j) const { return dbase + t + j; }

  // One tile operation of the inversion, (kind, i, j, k) in the paper's
  // naming, emitted with its hazard names and its device operands.  The
  // hazard names (reads/writes) are always the paper's tiles; the device may
  // read a different tile that holds the same values (a renaming copy, or
  // D_j / D_j^T for the inverted diagonal tile), which is safe when that tile
  // is written by the same task that is the last writer of the paper's tile
  // before the reader.  In the renamed plan every product reads op(A) = A and
  // op(B) = B^T contiguously (the copies are stored transposed); the in-place
  // plan uses the paper's tiles with transposes and triangular masks.
  // With partial renaming each operation takes the renamed form when the
  // tile row that holds its copy operands is renamed (B: the row of the L
  // tile read; C: the row of the X tiles read), the in-place form otherwise.
  void op(int kind, int i, int j, int k) {
    switch (kind) {
      // step 1, the Cholesky factor
      case K_SYRK1:   // A_jj -= A_jk A_jk^T
        emit(kind, j, j, k, {A(j, k), A(j, j)}, {A(j, j)}, A(j, j), A(j, k), A(j, k), -1, -1,
             F_TB | F_LOWER | F_NEG | F_ACC);
        break;
      case K_POTRF:   // A_jj <- chol(A_jj), D_j <- its inverse (B_jj <- the factor)
        if (rb(j)) emit(kind, j, j, 0, {A(j, j)}, {A(j, j), B(j, j)}, A(j, j), -1, -1, Bd(j, j), D(j));
        else emit(kind, j, j, 0, {A(j, j)}, {A(j, j)}, A(j, j), -1, -1, -1, D(j));
        break;
      case K_GEMM1:   // A_ij -= A_ik A_jk^T
        emit(kind, i, j, k, {A(i, k), A(j, k), A(i, j)}, {A(i, j)}, A(i, j), A(i, k), A(j, k), -1,
             -1, F_TB | F_NEG | F_ACC);
        break;
      case K_TRSM1:   // A_ij <- A_ij L_jj^{-T} = A_ij D_j^T (B_ij <- the result)
        emit(kind, i, j, 0, {A(j, j), A(i, j)}, rb(i) ? std::initializer_list<int>{A(i, j), B(i, j)}
                                                      : std::initializer_list<int>{A(i, j)},
             A(i, j), A(i, j), D(j), rb(i) ? Bd(i, j) : -1, -1, F_TB | (rb(i) ? F_COPYT : 0));
        break;
      // step 2, the inverse X = L^{-1}
      case K_TRTRI:   // A_jj <- D_j (and C_jj <- D_j^T)
        if (rc(j)) emit(kind, j, j, 0, {A(j, j)}, {A(j, j), C(j, j)}, A(j, j), D(j), Dt(j), Cd(j, j), -1);
        else emit(kind, j, j, 0, {A(j, j)}, {A(j, j)}, A(j, j), D(j), -1, -1, -1);
        break;
      case K_TRMM2L:  // A_ij <- X_ii L_ij
        if (rb(i))
          emit(kind, i, j, 0, {A(i, i), A(i, j)}, {A(i, j)}, A(i, j), A(i, i), Bd(i, j), -1, -1, F_TB);
        else
          emit(kind, i, j, 0, {A(i, i), A(i, j)}, {A(i, j)}, A(i, j), A(i, i), A(i, j), -1, -1, F_MA);
        break;
      case K_GEMM2:   // A_ij += X_ik L_kj
        if (rb(k))
          emit(kind, i, j, k, {A(i, k), B(k, j), A(i, j)}, {A(i, j)}, A(i, j), A(i, k), Bd(k, j), -1,
               -1, F_TB | F_ACC);
        else
          emit(kind, i, j, k, {A(i, k), A(k, j), A(i, j)}, {A(i, j)}, A(i, j), A(i, k), A(k, j), -1,
               -1, F_ACC);
        break;
      case K_TRSM2R: {  // A_ij <- -A_ij L_jj^{-1} = -A_ij D_j (C_ij <- the result)
        // by L_jj (a solve) in the LAPACK order, by X_jj after TRTRI(j) otherwise
        const int djj = (o.trtri_first || !rb(j)) ? A(j, j) : B(j, j);
        emit(kind, i, j, 0, {djj, A(i, j)}, rc(i) ? std::initializer_list<int>{A(i, j), C(i, j)}
                                                  : std::initializer_list<int>{A(i, j)},
             A(i, j), A(i, j), Dt(j), rc(i) ? Cd(i, j) : -1, -1,
             F_TB | F_NEG | (rc(i) ? F_COPYT : 0));
        break;
      }
      // step 3, the product X^T X
      case K_TRMM3:   // A_ij <- X_ii^T A_ij
        if (rc(i))
          emit(kind, i, j, 0, {C(i, i), A(i, j)}, {A(i, j)}, A(i, j), Cd(i, i), Cd(i, j), -1, -1, F_TB);
        else
          emit(kind, i, j, 0, {A(i, i), A(i, j)}, {A(i, j)}, A(i, j), A(i, i), A(i, j), -1, -1,
               F_TA | F_MA);
        break;
      case K_LAUUM:   // A_ii <- A_ii^T A_ii (lower)
        if (rc(i))
          emit(kind, i, i, 0, {A(i, i)}, {A(i, i)}, A(i, i), Cd(i, i), Cd(i, i), -1, -1,
               F_TB | F_LOWER);
        else
          emit(kind, i, i, 0, {A(i, i)}, {A(i, i)}, A(i, i), A(i, i), A(i, i), -1, -1,
               F_TA | F_MA | F_MB | F_LOWER);
        break;
      case K_GEMM3:   // A_ij += X_ki^T X_kj
        if (rc(k))
          emit(kind, i, j, k, {C(k, i), C(k, j), A(i, j)}, {A(i, j)}, A(i, j), Cd(k, i), Cd(k, j), -1,
               -1, F_TB | F_ACC);
        else
          emit(kind, i, j, k, {A(k, i), A(k, j), A(i, j)}, {A(i, j)}, A(i, j), A(k, i), A(k, j), -1,
               -1, F_TA | F_ACC);
        break;
      case K_SYRK3:   // A_ii += X_ki^T X_ki (lower)
        if (rc(k))
          emit(kind, i, i, k, {C(k, i), A(i, i)}, {A(i, i)}, A(i, i), Cd(k, i), Cd(k, i), -1, -1,
               F_TB | F_LOWER | F_ACC);
        else
          emit(kind, i, i, k, {A(k, i), A(i, i)}, {A(i, i)}, A(i, i), A(k, i), A(k, i), -1, -1,
               F_TA | F_LOWER | F_ACC);
        break;
      default:
        break;
    }
  }

  // The three steps as recurrences over output tiles (Algorithm 1; the
  // order of the updates of each tile is the paper's, and the tiles are
  // visited so that every operand a tile's recurrence reads is final
  // before the recurrence that reads it is emitted, except the tiles that
  // the paper's own order also reads before rewriting them -- which the
  // hazard analysis turns into anti-dependences).  Each tile's work is
  // emitted as one run: an optional opening operation, its update chain,
  // an optional closing operation.  The hazard DAG is that of the paper's
  // stream: per tile the accesses come in the same order.

  // Step 1: tile column j of L is final once column j's tiles have taken
  // the updates from every earlier column: the diagonal tile j its SYRKs
  // over k < j, then POTRF; each tile (i, j) below it its GEMMs over k < j,
  // then the solve with the factored diagonal tile.  Columns left to right.
  void step1() {
    cur_step = 1;
    for (int j = 0; j < t; ++j)
      for (int i = j; i < t; ++i) {
        const bool diag = i == j;
        for (int k = 0; k < j; ++k) op(diag ? K_SYRK1 : K_GEMM1, i, j, k);
        op(diag ? K_POTRF : K_TRSM1, i, j, 0);
      }
  }

  // Step 2: X_ij = -(X_ii L_ij + sum_{j<k<i} X_ik L_kj) L_jj^{-1} for i > j,
  // X_jj = L_jj^{-1}.  Columns right to left, rows bottom up, so that every
  // X_ik (k > j) a tile of column j reads is final; a tile's recurrence
  // opens with the product by X_ii, accumulates the chain over k (downward
  // in the UDU order, upward in UUU) and closes with the multiplication by
  // L_jj^{-1}.  The diagonal tile of the column is inverted after its
  // column (LAPACK order, reading L_jj) or before it (trtri_first, reading
  // X_jj).  With tree levels, the chain's sum is reassociated (the
  // associativity the conclusion, Section 4, points to) into segments run
  // side by side.
  void step2() {
    cur_step = 2;
    const bool down = (o.loop_order == 0);  // UDU: step-2 chain runs downward
    for (int j = t - 1; j >= 0; --j) {
      if (o.trtri_first) op(K_TRTRI, j, j, 0);
      for (int i = t - 1; i > j; --i) {
        op(K_TRMM2L, i, j, 0);
        const int m = i - j - 1;
        auto kk = [&](int s) { return down ? i - 1 - s : j + 1 + s; };
        if (!zper || m < 2) {
          for (int s = 0; s < m; ++s) op(K_GEMM2, i, j, kk(s));
        } else {
          // the chain cut into segs consecutive ranges of k (as equal as
          // possible, none empty), each in the loop order: segment l >= 1
          // (larger k, whose X_ik are final earlier) into its partial sum
          // Z_l, the partial sums added into A_ij in a fixed binary tree,
          // then segment 0 (k from j + 1, the last tiles to become final)
          // straight into A_ij, so that the chain's tail stays where the
          // sequential chain has it
          const int segs = std::min(zper + 1, m);
          auto terms = [&](int l, auto f) {
            const int k0 = j + 1 + (int)((long long)m * l / segs);
            const int k1 = j + 1 + (int)((long long)m * (l + 1) / segs);
            if (down)
              for (int k = k1 - 1; k >= k0; --k) f(k, k == k1 - 1);
            else
              for (int k = k0; k < k1; ++k) f(k, k == k0);
          };
          for (int l = 1; l < segs; ++l)
            terms(l, [&](int k, bool first) { gemm2_partial(i, j, k, l, first); });
          auto add = [&](int dst, int src) {
            if (dst == 0)
              emit(K_TADD, i, j, src, {Zh(i, j, src), A(i, j)}, {A(i, j)}, A(i, j), Zd(i, j, src),
                   -1, -1, -1, F_ACC);
            else
              emit(K_TADD, i, j, src, {Zh(i, j, src), Zh(i, j, dst)}, {Zh(i, j, dst)},
                   Zd(i, j, dst), Zd(i, j, src), -1, -1, -1, F_ACC);
          };
          if (segs == 2) {
            add(0, 1);
          } else if (segs == 3) {
            add(1, 2);
            add(0, 1);
          } else {
            add(1, 2);
            add(0, 3);
            add(0, 1);
          }
          terms(0, [&](int k, bool) { op(K_GEMM2, i, j, k); });
        }
        op(K_TRSM2R, i, j, 0);
      }
      if (!o.trtri_first) op(K_TRTRI, j, j, 0);
    }
  }

  // One term X_ik L_kj of the chain of tile (i, j) into its partial sum Z_l
  // (the first term of a segment overwrites it), in the form op() gives the
  // renamed or in-place step-2 product.
  void gemm2_partial(int i, int j, int k, int l, bool first) {
    const int acc = first ? 0 : F_ACC;
    if (rb(k))
      emit(K_GEMM2, i, j, k, {A(i, k), B(k, j), Zh(i, j, l)}, {Zh(i, j, l)}, Zd(i, j, l), A(i, k),
           Bd(k, j), -1, -1, F_TB | acc);
    else
      emit(K_GEMM2, i, j, k, {A(i, k), A(k, j), Zh(i, j, l)}, {Zh(i, j, l)}, Zd(i, j, l), A(i, k),
           A(k, j), -1, -1, acc);
  }

  // Step 3: (X^T X)_ij = sum_{k >= i} X_ki^T X_kj for i >= j.  Rows top down;
  // in row i the tiles left of the diagonal, then the diagonal tile: each
  // opens with its k = i term (the product by X_ii^T, or LAUUM on the
  // diagonal) and accumulates the terms k > i upward.  (In place, X_ii is
  // still read by the row's first products when LAUUM overwrites it, which
  // is why the diagonal tile comes last in its row.)
  void step3() {
    cur_step = 3;
    for (int i = 0; i < t; ++i)
      for (int j = 0; j <= i; ++j) {
        const bool diag = i == j;
        op(diag ? K_LAUUM : K_TRMM3, i, j, 0);
        for (int k = i + 1; k < t; ++k) op(diag ? K_SYRK3 : K_GEMM3, i, j, k);
      }
  }

  // The solve A X = R with A = L L^T, over the s tile columns of R: forward
  // substitution L Y = R (row i: R_ic -= L_ik Y_kc for k = 0..i-1, then Y_ic =
  // D_i R_ic), then backward L^T X = Y (row i from the last: R_ic -= L_ki^T
  // X_kc for k = t-1 down to i+1, then X_ic = D_i^T R_ic).  The explicit
  // diagonal inverses D_i replace the triangular solves with the diagonal
  // tiles, as in steps 1 and 2.  The right-hand-side tiles are kept
  // transposed (tile (i, c) holds R_ic^T), so that every product has the
  // column form C -= A B^T of the renamed plan: R_ic^T -= R_kc^T L_ik^T,
  // R_ic^T <- R_ic^T D_i^T, R_ic^T -= R_kc^T L_ki (B = the renaming copy
  // L_ki^T), R_ic^T <- R_ic^T D_i (B = D_i^T); the in-place plan reads L_ki
  // untransposed instead.
  void solve() {
    cur_step = 4;
    const int s = o.rhs_tiles;
    for (int i = 0; i < t; ++i)
      for (int c = 0; c < s; ++c) {
        for (int k = 0; k < i; ++k)
          emit(K_GEMMS, i, c, k, {A(i, k), Rh(k, c), Rh(i, c)}, {Rh(i, c)}, Rp(i, c), Rp(k, c),
               A(i, k), -1, -1, F_TB | F_NEG | F_ACC);
        emit(K_TRSMS, i, c, 0, {A(i, i), Rh(i, c)}, {Rh(i, c)}, Rp(i, c), Rp(i, c), D(i), -1, -1,
             F_TB);
      }
    for (int i = t - 1; i >= 0; --i)
      for (int c = 0; c < s; ++c) {
        for (int k = t - 1; k > i; --k) {
          if (rb(k))
            emit(K_GEMMS, i, c, k, {B(k, i), Rh(k, c), Rh(i, c)}, {Rh(i, c)}, Rp(i, c), Rp(k, c),
                 Bd(k, i), -1, -1, F_TB | F_NEG | F_ACC);
          else
            emit(K_GEMMS, i, c, k, {A(k, i), Rh(k, c), Rh(i, c)}, {Rh(i, c)}, Rp(i, c), Rp(k, c),
                 A(k, i), -1, -1, F_NEG | F_ACC);
        }
        emit(K_TRSMS, i, c, 0, {A(i, i), Rh(i, c)}, {Rh(i, c)}, Rp(i, c), Rp(i, c), Dt(i), -1, -1,
             F_TB);
      }
  }
};

inline int weight(int kind) { return task_kind(kind) == K_NOP ? 0 : 1; }

// Emits the task stream of the options' steps (as build_plan does).
void emit_stream(Builder& bld, const PlanOptions& opt) {
  const bool s1 = opt.steps & 1, s2 = opt.steps & 2, s3 = opt.steps & 4;
  if (s1) bld.step1();
  if (s1 && (s2 || s3) && !opt.pipelined) bld.emit_barrier();
  if (s2) bld.step2();
  if (s2 && s3 && !opt.pipelined) bld.emit_barrier();
  if (s3) bld.step3();
  if (opt.steps & 8) {
    if (s1 && !opt.pipelined) bld.emit_barrier();
    bld.solve();
  }
}

// List-scheduling simulation of a DAG given by predecessor lists in a
// topological program order: `workers` identical workers, priority =
// weighted bottom level (longest remaining path), ties broken by program
// order.  Returns the dispatch order and, if asked, each task's simulated
// start time.
void list_schedule(const std::vector<std::vector<int32_t>>& preds, const std::vector<double>& dur,
                   int workers, std::vector<int32_t>* order, std::vector<double>* start) {
  const int n = (int)preds.size();
  std::vector<int32_t> ptr(n + 1, 0), deg(n, 0);
  for (int v = 0; v < n; ++v)
    for (int q : preds[v]) ptr[q + 1]++;
  for (int v = 0; v < n; ++v) ptr[v + 1] += ptr[v];
  std::vector<int32_t> succ(ptr[n]);
  {
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int v = 0; v < n; ++v) {
      deg[v] = (int32_t)preds[v].size();
      for (int q : preds[v]) succ[fill[q]++] = v;
    }
  }
  std::vector<double> bl(n, 0.0);
  for (int v = n - 1; v >= 0; --v) {
    double m = 0.0;
    for (int e = ptr[v]; e < ptr[v + 1]; ++e) m = std::max(m, bl[succ[e]]);
    bl[v] = dur[v] + m;
  }
  auto cmp = [&](int x, int y) {  // max-heap on bl, then min program index
    if (bl[x] != bl[y]) return bl[x] < bl[y];
    return x > y;
  };
  std::priority_queue<int, std::vector<int>, decltype(cmp)> ready(cmp);
  using Ev = std::pair<double, int>;
  std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> running;
  for (int v = 0; v < n; ++v)
    if (deg[v] == 0) ready.push(v);
  if (order) {
    order->clear();
    order->reserve(n);
  }
  if (start) start->assign(n, 0.0);
  double now = 0.0;
  int busy = 0, done = 0;
  const int P = std::max(1, workers);
  while (done < n) {
    while (busy < P && !ready.empty()) {
      const int v = ready.top();
      ready.pop();
      if (order) order->push_back(v);
      if (start) (*start)[v] = now;
      running.push({now + dur[v], v});
      ++busy;
    }
    if (running.empty()) break;  // cannot happen for an acyclic plan
    now = running.top().first;
    while (!running.empty() && running.top().first <= now) {
      const int v = running.top().second;
      running.pop();
      --busy;
      ++done;
      for (int e = ptr[v]; e < ptr[v + 1]; ++e)
        if (--deg[succ[e]] == 0) ready.push(succ[e]);
    }
  }
}

// A product that reads both operands along stored columns (op(A) = A,
// op(B) = B^T, no masks): the form the chained device product executes.
bool column_product(const DevTask& d) {
  const int k = task_kind(d.kind);
  if (k == K_NOP || k == K_POTRF || k == K_TRTRI || k == K_TADD) return false;
  const int f = task_flags(d.kind);
  return (f & (F_TA | F_MA | F_MB)) == 0 && (f & F_TB) != 0;
}

// v can continue the chain of u: the next product on u's output tile,
// accumulating, with the same sign and output mask, operands other than the
// output tile, and no renaming copy of u's (intermediate) result.
bool chainable(const DevTask& u, const DevTask& v) {
  if (!column_product(u) || !column_product(v)) return false;
  const int fu = task_flags(u.kind), fv = task_flags(v.kind);
  return u.copy < 0 && (fv & F_ACC) && ((fu ^ fv) & (F_NEG | F_LOWER)) == 0 && v.a != v.out &&
         v.b != v.out;
}

// Contracts runs of consecutive products of one output tile into device
// tasks of at most `chain` links.  A run is extended by v only if
//  - every predecessor of v other than the previous link comes before the
//    run's head in program order (so the contracted DAG stays acyclic and
//    program order stays topological);
//  - v is not the last product of its chain (the one followed by a
//    non-chainable writer of the tile, or by none): that product waits for
//    the most recently finished operand, so it stays a task of its own
//    (unless `tails`: a plan run in order by one workgroup);
//  - in the simulated schedule of the uncontracted DAG (start times `st`,
//    durations `dur`, `link` per further link), v's other predecessors have
//    finished by the time the contracted task would reach v, give or take
//    `slack`, so contraction delays the head by at most that much.  (On
//    MI355X at n = 8192, a slack of 5 single-product durations made chain
//    lengths 6 to 12 equally fast; without the rule, lengths above 8 held
//    early tasks back and lost up to 20 %.)
// The contracted task sits at the head's position; its predecessors are the
// union of the members' external predecessors.
void chain_products(int chain, Plan* p, std::vector<std::vector<int32_t>>& preds,
                    const std::vector<double>& st, const std::vector<double>& dur, double link,
                    double slack, bool tails) {
  const int n = (int)p->tasks.size();
  std::vector<int32_t> next_out(n, -1);
  {
    std::unordered_map<int32_t, int32_t> last;
    for (int v = n - 1; v >= 0; --v) {
      const int o = p->tasks[v].out;
      if (o < 0) continue;
      auto it = last.find(o);
      next_out[v] = it == last.end() ? -1 : it->second;
      last[o] = v;
    }
  }
  auto tail = [&](int v) {  // v is the last product of its chain (and must run alone)
    if (tails) return false;
    const int w = next_out[v];
    return w < 0 || !chainable(p->tasks[v], p->tasks[w]);
  };
  std::vector<int32_t> head(n, -1);  // contracted task of each member
  std::vector<std::vector<int32_t>> members(n);
  for (int u = 0; u < n; ++u) {
    if (head[u] >= 0) continue;
    head[u] = u;
    members[u].push_back(u);
    if (!column_product(p->tasks[u]) || tail(u)) continue;
    int last = u;
    while ((int)members[u].size() < chain) {
      const int v = next_out[last];
      if (v < 0 || !chainable(p->tasks[last], p->tasks[v]) || tail(v) || head[v] >= 0) break;
      // the contracted task reaches link m = members.size() at this time
      const double reach = st[u] + dur[u] + link * (double)(members[u].size() - 1);
      bool early = true;
      for (int q : preds[v])
        if (q != last && (q >= u || st[q] + dur[q] > reach + slack)) { early = false; break; }
      if (!early) break;
      head[v] = u;
      members[u].push_back(v);
      last = v;
    }
  }
  std::vector<int32_t> pos(n, -1);
  int m = 0;
  for (int u = 0; u < n; ++u)
    if (head[u] == u) pos[u] = m++;
  std::vector<DevTask> tasks;
  std::vector<int32_t> step, idx;
  std::vector<std::vector<int32_t>> np;
  tasks.reserve(m);
  step.reserve(m);
  idx.reserve(m);
  np.reserve(m);
  p->links.clear();
  for (int u = 0; u < n; ++u) {
    if (head[u] != u) continue;
    const std::vector<int32_t>& mem = members[u];
    DevTask d = p->tasks[u];
    if (mem.size() > 1) {
      const DevTask& z = p->tasks[mem.back()];
      d.copy = z.copy;
      d.kind = (d.kind & ~(F_COPYT << 8)) | (z.kind & (F_COPYT << 8));
      d.kind |= (int32_t)(mem.size() - 1) << K_LINKS_SHIFT;
      // the chained product reads every operand device-coherent
      d.kind &= ~(K_NC_A | K_NC_B);
      d.aux = (int32_t)(p->links.size() / 2);
      for (size_t q = 1; q < mem.size(); ++q) {
        const DevTask& e = p->tasks[mem[q]];
        p->links.push_back(e.a | ((e.kind & K_KLAST) ? LINK_KLAST : 0));
        p->links.push_back(e.b);
      }
    }
    std::vector<int32_t> pr;
    for (int x : mem)
      for (int q : preds[x])
        if (head[q] != u) pr.push_back(pos[head[q]]);
    std::sort(pr.begin(), pr.end());
    pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
    tasks.push_back(d);
    step.push_back(p->step[u]);
    idx.push_back(p->idx[u]);
    np.push_back(std::move(pr));
  }
  p->tasks.swap(tasks);
  p->step.swap(step);
  p->idx.swap(idx);
  preds.swap(np);
}

}  // namespace

// Splits the single column-form products of the chains of dependent tasks
// into `parts` row-part tasks (K_PART, 2 or 4): between POTRF(j) and POTRF(j+1), TRSM(j+1, j)
// and the last SYRK into tile (j+1, j+1); in the solve, each multiplication
// by D_i or D_i^T and the last update of its right-hand-side tile before it
// (each row's pair waits for the previous row's).  Both halves take the
// product's predecessors, every successor of the product waits for all of
// them, and the parts follow each other in program order (which stays
// topological).
// Duration of a device task in the dispatch cost model: `cost` per kind
// and per further chain link (else unit weights); a row half costs
// cost[K_COUNT + 1] of the whole product, a quarter 0.75 of that.
double model_duration(int32_t k, const double* cost) {
  double d = cost ? cost[task_kind(k)] + cost[K_COUNT] * task_links(k)
                  : (double)weight(k) * (1 + task_links(k));
  if (k & K_PART)
    d *= cost ? cost[K_COUNT + 1] * ((k & K_PARTS4) ? 0.75 : 1.0) : ((k & K_PARTS4) ? 0.25 : 0.5);
  return d;
}

// Slack of every task in the cost model: the critical path minus the
// longest path through the task (earliest start plus longest remaining
// path).  Tasks are in a topological program order.
std::vector<double> model_slack(const Plan& p, const std::vector<std::vector<int32_t>>& preds,
                                const double* cost) {
  const int n = (int)p.tasks.size();
  std::vector<double> dur(n), tl(n, 0.0), best(n, 0.0), bl(n, 0.0);
  for (int v = 0; v < n; ++v) dur[v] = model_duration(p.tasks[v].kind, cost);
  for (int v = 0; v < n; ++v)
    for (int q : preds[v]) tl[v] = std::max(tl[v], tl[q] + dur[q]);
  double cpl = 0.0;
  for (int v = n - 1; v >= 0; --v) {  // successors have larger indices
    bl[v] = dur[v] + best[v];
    for (int q : preds[v]) best[q] = std::max(best[q], bl[v]);
    cpl = std::max(cpl, tl[v] + bl[v]);
  }
  std::vector<double> slack(n);
  for (int v = 0; v < n; ++v) slack[v] = cpl - (tl[v] + bl[v]);
  return slack;
}

void split_critical_products(Plan* p, std::vector<std::vector<int32_t>>& preds, int parts) {
  const int n = (int)p->tasks.size();
  auto single = [&](int v) {
    const DevTask& d = p->tasks[v];
    return column_product(d) && task_links(d.kind) == 0 && !(d.kind & K_PART);
  };
  std::vector<char> mark(n, 0);
  for (int v = 0; v < n; ++v) {
    const DevTask& ts = p->tasks[v];
    if (task_kind(ts.kind) != K_TRSMS || !single(v)) continue;
    mark[v] = 1;
    for (int q : preds[v]) {
      const DevTask& up = p->tasks[q];
      if (task_kind(up.kind) == K_GEMMS && up.out == ts.out && single(q)) mark[q] = 1;
    }
  }
  for (int v = 0; v < n; ++v) {
    const DevTask& pot = p->tasks[v];
    if (task_kind(pot.kind) != K_POTRF) continue;
    for (int q : preds[v]) {
      const DevTask& sy = p->tasks[q];
      if (task_kind(sy.kind) != K_SYRK1 || sy.out != pot.out || !single(q)) continue;
      mark[q] = 1;
      for (int r : preds[q]) {
        const DevTask& tr = p->tasks[r];
        if (task_kind(tr.kind) == K_TRSM1 && tr.out == sy.a && single(r)) mark[r] = 1;
      }
    }
  }
  std::vector<int32_t> first(n), count(n, 1);
  int m = 0;
  for (int v = 0; v < n; ++v) {
    first[v] = m;
    if (mark[v]) count[v] = parts;
    m += count[v];
  }
  if (m == n) return;
  std::vector<DevTask> tasks(m);
  std::vector<int32_t> step(m), idx(m);
  std::vector<std::vector<int32_t>> np(m);
  for (int v = 0; v < n; ++v) {
    std::vector<int32_t> pv;
    pv.reserve(preds[v].size() + 2);
    for (int q : preds[v])
      for (int c = 0; c < count[q]; ++c) pv.push_back(first[q] + c);
    for (int c = 0; c < count[v]; ++c) {
      const int u = first[v] + c;
      tasks[u] = p->tasks[v];
      if (mark[v])
        tasks[u].kind |= K_PART | (c << K_PART_SHIFT) | (parts == 4 ? K_PARTS4 : 0);
      step[u] = p->step[v];
      idx[u] = p->idx[v];
      np[u] = pv;
    }
  }
  p->tasks.swap(tasks);
  p->step.swap(step);
  p->idx.swap(idx);
  preds.swap(np);
}

void build_plan(const PlanOptions& opt, int workers, const double* cost, Plan* p) {
  *p = Plan();
  p->opt = opt;
  const int t = opt.t;
  p->T = t * (t + 1) / 2;
  Builder bld(opt, p);
  emit_stream(bld, opt);

  // dead factor stores: a POTRF whose factor tile is not read before it is
  // rewritten, and whose renaming copy is never read, stores only D_j, D_j^T.
  // A tile that no later task rewrites holds a final value (the copy-out
  // reads it).  Renaming copies that no task reads are not stored either.
  {
    const int nt = (int)p->tasks.size();
    std::vector<char> copy_read(p->pool_tiles, 0);
    for (const DevTask& d : p->tasks) {
      if (d.a >= 0) copy_read[d.a] = 1;
      if (d.b >= 0) copy_read[d.b] = 1;
    }
    for (int u = 0; u < nt; ++u) {
      DevTask& d = p->tasks[u];
      if (task_kind(d.kind) != K_POTRF) continue;
      bool read = d.copy >= 0 && copy_read[d.copy];
      bool rewritten = false;
      for (int v = u + 1; v < nt && !read; ++v) {
        const DevTask& e = p->tasks[v];
        if (task_kind(e.kind) == K_NOP) continue;
        if (e.a == d.out || e.b == d.out) read = true;
        if (e.out == d.out) {  // next writer: an accumulating product reads it first
          if (task_flags(e.kind) & F_ACC) read = true;
          rewritten = true;
          break;
        }
      }
      if (!rewritten) read = true;  // final value of the tile
      if (!read) {
        d.kind |= K_POTRF_FACTOR_DEAD;
        d.copy = -1;
      }
      if (d.aux >= 0 && !copy_read[d.aux + p->opt.t]) d.kind |= K_POTRF_INVT_DEAD;
    }
    for (int u = 0; u < nt; ++u) {
      DevTask& d = p->tasks[u];
      if (d.copy < 0 || copy_read[d.copy]) continue;
      d.copy = -1;
      d.kind &= ~(F_COPYT << 8);
    }
  }

  // L2-cacheable operand reads: only tiles written exactly once in the plan
  // and not accessed at all before that write (the renaming copies and the
  // inverted diagonal tiles).  Device-coherent loads may still leave lines
  // in the reading XCD's L2, so a tile that was read (or written) in an
  // earlier version during the launch is never read through the cache.
  {
    const int nt = (int)p->tasks.size();
    const int64_t ntiles = p->pool_tiles;
    std::vector<int32_t> writes(ntiles, 0);
    std::vector<char> touched_first(ntiles, 0);  // accessed before its first write
    for (int u = 0; u < nt; ++u) {
      const DevTask& d = p->tasks[u];
      const int k = task_kind(d.kind);
      if (k == K_NOP) continue;
      const bool acc = k != K_POTRF && k != K_TRTRI && (task_flags(d.kind) & F_ACC);
      for (int tile : {d.a, d.b}) {
        if (tile >= 0 && writes[tile] == 0) touched_first[tile] = 1;
      }
      if ((acc || k == K_POTRF) && d.out >= 0 && writes[d.out] == 0) touched_first[d.out] = 1;
      if (d.out >= 0) writes[d.out]++;
      if (d.copy >= 0) writes[d.copy]++;
      if (k == K_POTRF) {
        writes[d.aux]++;
        writes[d.aux + opt.t]++;
      }
    }
    auto cacheable = [&](int tile) {
      return tile >= 0 && writes[tile] == 1 && !touched_first[tile];
    };
    for (int u = 0; u < nt; ++u) {
      DevTask& d = p->tasks[u];
      const int k = task_kind(d.kind);
      if (k == K_NOP || k == K_POTRF || k == K_TRTRI || k == K_TADD) continue;
      if (cacheable(d.a)) d.kind |= K_NC_A;
      if (cacheable(d.b)) d.kind |= K_NC_B;
    }
  }

  // products whose reduction index is the last tile block: the stored
  // columns of a pool tile are its column block for A tiles and D_j, its row
  // block for the transposed copies B, C and D_j^T
  {
    const int T = p->T;
    const int last = t - 1;
    auto in_row = [&](int base, int x) { return base >= 0 && x >= base && x < base + t; };
    auto klast = [&](int x) {
      if (x < 0) return false;
      if (x < T) return x == T - 1;                                      // A(t-1, t-1)
      if (x < bld.dbase) return in_row(bld.boff[last], x) || in_row(bld.coff[last], x);
      return x == bld.dbase + t - 1 || x == bld.dbase + 2 * t - 1;      // D_{t-1}, D_{t-1}^T
    };
    for (DevTask& d : p->tasks)
      if (column_product(d) && (klast(d.a) || klast(d.b))) d.kind |= K_KLAST;
  }

  // statistics of the paper's DAG: task counts and critical paths (unit
  // weight per task)
  {
    const int n = (int)p->tasks.size();
    PlanStats& st = p->stats;
    std::memset(&st, 0, sizeof(st));
    st.ntasks = n;
    for (int v = 0; v < n; ++v) {
      st.nedges += (int64_t)bld.preds[v].size();
      st.count[task_kind(p->tasks[v].kind)]++;
    }
    std::vector<int32_t> lp(n, 0), ls(n, 0);
    int cp = 0, cps[5] = {0, 0, 0, 0, 0};  // by step (0 = barriers, 4 = the solve)
    for (int v = 0; v < n; ++v) {  // program order is a topological order
      int best = 0, best_s = 0;
      for (int q : bld.preds[v]) {
        best = std::max(best, lp[q]);
        if (p->step[q] == p->step[v]) best_s = std::max(best_s, ls[q]);
      }
      lp[v] = best + weight(p->tasks[v].kind);
      ls[v] = best_s + weight(p->tasks[v].kind);
      cp = std::max(cp, lp[v]);
      cps[p->step[v]] = std::max(cps[p->step[v]], ls[v]);
    }
    st.cp_step[0] = cps[1];
    st.cp_step[1] = cps[2];
    st.cp_step[2] = cps[3];
    st.cp_unpipelined = cps[1] + cps[2] + cps[3];
    st.cp_plan = cp;
    st.cp_pipelined = opt.pipelined ? cp : -1;
  }

  if (opt.chain > 1) {
    const int n0 = (int)p->tasks.size();
    std::vector<double> dur0(n0), st0;
    for (int v = 0; v < n0; ++v)
      dur0[v] = cost ? cost[task_kind(p->tasks[v].kind)] : (double)weight(p->tasks[v].kind);
    list_schedule(bld.preds, dur0, workers, nullptr, &st0);
    // slack: 5 single-product durations (the unit of `cost`)
    chain_products(opt.chain, p, bld.preds, st0, dur0, cost ? cost[K_COUNT] : 1.0, 5.0,
                   opt.chain_tails != 0);
  }
  if (opt.split == 2 || opt.split == 4) split_critical_products(p, bld.preds, opt.split);

  const int n = (int)p->tasks.size();
  // CSR successors
  std::vector<int32_t> outdeg(n, 0);
  int64_t ne = 0;
  p->indeg.assign(n, 0);
  for (int v = 0; v < n; ++v) {
    p->indeg[v] = (int32_t)bld.preds[v].size();
    for (int q : bld.preds[v]) outdeg[q]++;
    ne += (int64_t)bld.preds[v].size();
  }
  std::vector<int32_t> ptr(n + 1, 0);
  for (int v = 0; v < n; ++v) ptr[v + 1] = ptr[v] + outdeg[v];
  p->succ.assign(ne, 0);
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  for (int v = 0; v < n; ++v)
    for (int q : bld.preds[v]) p->succ[fill[q]++] = v;
  for (int v = 0; v < n; ++v) {
    p->tasks[v].succ_begin = ptr[v];
    p->tasks[v].succ_end = ptr[v + 1];
  }

  // dispatch order: list-scheduling simulation of the executed DAG
  // (a row half costs cost[K_COUNT + 1] of the whole product, a quarter
  // 0.75 of that)
  std::vector<double> dur(n);
  for (int v = 0; v < n; ++v) dur[v] = model_duration(p->tasks[v].kind, cost);
  // near-critical tasks (K_URGENT): slack under half a single product
  {
    const std::vector<double> slack = model_slack(*p, bld.preds, cost);
    const double eps = 0.5 * (cost ? cost[K_COUNT] : 1.0);
    for (int v = 0; v < n; ++v)
      if (dur[v] > 0.0 && slack[v] < eps) p->tasks[v].kind |= K_URGENT;
  }
  list_schedule(bld.preds, dur, workers, &p->order, nullptr);
}

int renamed_tiles(const PlanOptions& opt) {
  if (!opt.renamed) return 0;
  int n = 0;
  for (int i = 0; i < opt.t; ++i) {
    if (opt.ren_b.empty() || opt.ren_b[i]) n += i + 1;
    if (opt.ren_c.empty() || opt.ren_c[i]) n += i + 1;
  }
  return n;
}

int plan_critical_path(const PlanOptions& opt) {
  Plan p;
  p.opt = opt;
  p.T = opt.t * (opt.t + 1) / 2;
  Builder bld(opt, &p);
  emit_stream(bld, opt);
  const int n = (int)p.tasks.size();
  std::vector<int32_t> lp(n, 0);
  int cp = 0;
  for (int v = 0; v < n; ++v) {
    int best = 0;
    for (int q : bld.preds[v]) best = std::max(best, lp[q]);
    lp[v] = best + weight(p.tasks[v].kind);
    cp = std::max(cp, lp[v]);
  }
  return cp;
}

void choose_renaming(PlanOptions* opt, long long budget) {
  const int t = opt->t;
  opt->ren_b.clear();
  opt->ren_c.clear();
  if (!opt->renamed || budget >= (long long)t * (t + 1)) return;  // full renaming
  opt->ren_b.assign(t, 0);
  opt->ren_c.assign(t, 0);
  long long left = budget;
  // the critical path of every candidate is evaluated up to 16 tiles per
  // side (a round costs 2t builds of the t^3/2-task stream); beyond, rows
  // are taken in the fallback order, which reaches the same critical paths
  // where both were compared (8 to 32 tiles per side)
  const bool evaluate = t <= 16;
  int cp = evaluate ? plan_critical_path(*opt) : 0;
  for (;;) {
    // candidate rows (copy, row), each costing row + 1 tiles
    int best_c = -1, best_r = -1;
    double best_score = 0.0;
    int best_cp = cp;
    for (int c = 0; c < 2 && evaluate; ++c)
      for (int r = 0; r < t; ++r) {
        std::vector<char>& v = c ? opt->ren_c : opt->ren_b;
        if (v[r] || r + 1 > left) continue;
        v[r] = 1;
        const int cpr = plan_critical_path(*opt);
        v[r] = 0;
        const double score = double(cp - cpr) / (r + 1);
        if (score > best_score) {
          best_score = score;
          best_c = c;
          best_r = r;
          best_cp = cpr;
        }
      }
    if (best_c < 0) {
      // no single row shortens the path (or the candidates are not
      // evaluated): the last C row, then the B rows from the top (a B row's
      // diagonal tile names the factor tile that the column's right solves
      // read before TRTRI rewrites it), then the C rows from the bottom --
      // the rows the evaluated greedy takes at 8 to 32 tiles per side
      if (!opt->ren_c[t - 1] && t <= left) {
        best_c = 1;
        best_r = t - 1;
      }
      for (int r = 0; r < t && best_c < 0; ++r)
        if (!opt->ren_b[r] && r + 1 <= left) {
          best_c = 0;
          best_r = r;
        }
      for (int r = t - 1; r >= 0 && best_c < 0; --r)
        if (!opt->ren_c[r] && r + 1 <= left) {
          best_c = 1;
          best_r = r;
        }
      if (best_c < 0) break;  // nothing fits
      std::vector<char>& v = best_c ? opt->ren_c : opt->ren_b;
      v[best_r] = 1;
      best_cp = evaluate ? plan_critical_path(*opt) : 0;
    } else {
      (best_c ? opt->ren_c : opt->ren_b)[best_r] = 1;
    }
    left -= best_r + 1;
    cp = best_cp;
  }
}

}  // namespace spdinv
