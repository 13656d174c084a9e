// Chebyshev-step kernels: Y = s1 (Htilde - shift) X + s2 Xprev with
// Htilde X = M^-1/2 (sum_e P_e^T K_e P_e) M^-1/2 X + V .* X.
//
// Paper, Sec. 3.3 (practical implementation of Chebyshev filtering): store the
// cell Hamiltonian, extract the cell wavefunction matrices from the DoF-major
// global block, multiply, assemble.  On a uniform mesh every cell carries the
// same stiffness K_ref, so the cell products form one dense contraction
// K_ref [n_loc x n_loc] x X_e [n_loc x ncols] per cell, done here on MFMA.
// Under GLL quadrature the potential part is diagonal.
//
// Assembly is atomic-free: cells are launched colour by colour (8 colours,
// (ex&1)+2(ey&1)+4(ez&1)); cells of one colour share no DoF, so each output
// row is touched by exactly one work-group per launch.  The element-wise part
// s1 (V - shift) X + s2 Xprev is fused into the first touch: colours run in
// increasing order, and the first colour containing a node is the one whose
// parity bit is 0 in every direction where the node lies on a cell face; the
// single cell of that colour containing the node writes Y (element-wise part
// plus its product), every later cell adds to Y.
#include "common.hpp"
#include "kernels.hpp"


namespace chfsi {

// 1 when this cell is the first (in colour order) to touch local node r
__device__ __forceinline__ int first_touch(int r, int q, int e, int n_el) {
  const int a = r % q, b = (r / q) % q, c = r / (q * q);
  const int ex = e % n_el, ey = (e / n_el) % n_el, ez = e / (n_el * n_el);
  const bool fx = (a > 0 && a < q - 1) || !(ex & 1);
  const bool fy = (b > 0 && b < q - 1) || !(ey & 1);
  const bool fz = (c > 0 && c < q - 1) || !(ez & 1);
  return (fx && fy && fz) ? 1 : 0;
}

// Epilogue of one 16-row x 16-column output fragment (4 rows per lane):
// Y[dof, col] = s1 (V - shift) X + s2 Xprev + s1 minv acc on the row's first
// touch, Y[dof, col] += s1 minv acc afterwards.  Loads and stores are split so
// that a caller issues the loads of the next fragment before it stores this
// one, and every load is unconditional (a row that is not written reads an
// in-bounds address), so no branch sits between a load and its consumer.
template <typename T>
struct EpiFrag {
  T v1[4], v2[4];
};

template <typename T>
struct EpiCtx {
  const T *X;
  int64_t ldx;
  const T *Xp;
  int64_t ldp;
  T *Y;
  int64_t ldy;
  const int32_t *dof_s;
  const T *mi_s, *vd_s;
  const int8_t *ft_s;
  int n_loc;
  T s1, s2;
};

template <typename T>
__device__ __forceinline__ void epi_load(const EpiCtx<T> &c, int row0, int kq, int col, EpiFrag<T> &f) {
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    const int row = row0 + acc_row<T>(kq, qq);
    const int64_t d = c.dof_s[row];
    const bool ft = c.ft_s[row] != 0;
    const T *p1 = ft ? c.X + d * c.ldx : c.Y + d * c.ldy;
    const T *p2 = (ft && c.Xp) ? c.Xp + d * c.ldp : p1;
    f.v1[qq] = p1[col];
    f.v2[qq] = p2[col];
  }
}

template <typename T, typename A>
__device__ __forceinline__ void epi_store(const EpiCtx<T> &c, int row0, int kq, int col, bool col_ok,
                                          const EpiFrag<T> &f, const A &acc) {
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    const int row = row0 + acc_row<T>(kq, qq);
    const T w = c.mi_s[row];
    if (col_ok && row < c.n_loc && w != T(0)) {
      const T prod = c.s1 * w * acc[qq];
      T y;
      if (c.ft_s[row]) {
        y = c.vd_s[row] * f.v1[qq] + prod;
        if (c.Xp) y += c.s2 * f.v2[qq];
      } else {
        y = f.v1[qq] + prod;
      }
      c.Y[(int64_t)c.dof_s[row] * c.ldy + col] = y;
    }
  }
}

// ---------------------------------------------------------------------------
// Cell products of one colour (FP64 and FP32), both operands staged through
// LDS.  Work-group = one cell x TW columns, NW waves in a WR x WC grid: wave (wr, wc)
// owns row blocks [wr*RBW, (wr+1)*RBW) and column blocks [wc*CBW, (wc+1)*CBW)
// of the 16x16 output tiles, so every A fragment read from LDS feeds CBW MFMAs
// and every B fragment RBW MFMAs.  The contraction index runs over chunks of
// KC local nodes: a chunk of K_ref (KC full rows, contiguous in the padded
// matrix) and of the gathered, M^-1/2-scaled X_e (KC rows x TW columns) is
// loaded into registers one chunk ahead, written to the other half of a
// double-buffered LDS area after the chunk's MFMAs, and published by the one
// barrier per chunk.  K_ref is thus read once per work-group, and each
// gathered row once per work-group.
// ---------------------------------------------------------------------------
template <typename T, int NP, int NW, int WR, int CBW, int KC>
struct LdsTile {
  static constexpr int NT = 64 * NW;                       // threads
  static constexpr int RB = NP / 16;
  static constexpr int RBW = RB / WR;
  static constexpr int WC = NW / WR;
  static constexpr int TW = 16 * CBW * WC;                 // columns per work-group
  static constexpr int VEC = 16 / sizeof(T);               // elements per 16-byte load
  static constexpr int KV = KC * NP / VEC;                 // 16-byte vectors per K chunk
  static constexpr int KPT = (KV + NT - 1) / NT;           // ... per thread
  static constexpr int XPT = KC * TW / NT;                 // X values per thread per chunk
  static constexpr int NCH = NP / KC;                      // chunks
  // LDS row strides.  A 64-lane FP32 fragment read touches four rows of 16
  // consecutive words; a stride of 16 (mod 32) words spreads them over both
  // halves of the 32 banks (no conflicts beyond the 2-cycle minimum).  FP64
  // reads take 4 cycles regardless, so FP64 rows stay unpadded.
  static constexpr int pad32(int n) { return sizeof(T) == 4 ? n + (48 - n % 32) % 32 : n; }
  static constexpr int SK = pad32(NP);
  static constexpr int SX = pad32(TW);
  static_assert(RB % WR == 0 && NW % WR == 0, "row blocks must split over the wave rows");
  static_assert(KC % 4 == 0 && NP % KC == 0 && (KC * NP) % VEC == 0, "chunking");
  static_assert((KC * TW) % NT == 0, "X chunk must split evenly over the threads");
  static_assert((SK * sizeof(T)) % 16 == 0, "16-byte LDS stores of K rows");
};

// CPLX: complex products on interleaved (re, im) columns with K = [A ; B^T]
// (2 NP rows): the contraction runs twice as long, and its second half
// gathers each column's partner (col ^ 1), negated for imaginary outputs, so
// Y_re = A Xr + B Xi and Y_im = A Xi - B Xr.
// CPT cells per work-group: the TW tile columns are split into CPT groups of
// CW = TW / CPT columns, group s holding columns [col0, col0 + CW) of cell
// ecells[s] (cells of one colour share no DoF, so their rows never collide);
// necell <= CPT of the slots are filled.  CPT = 1 is one cell x TW columns.
template <typename T, int NP, int NW, int WR, int CBW, int KC, int EPD, bool CPLX = false, int CPT = 1, int XD = 2>
__device__ __forceinline__ void cell_tile(const T *__restrict__ X, int64_t ldx, const T *__restrict__ Xp,
                                              int64_t ldp, T *__restrict__ Y, int64_t ldy,
                                              const T *__restrict__ K, const int32_t *__restrict__ cmap,
                                              int n_loc, int q, int n_el, const int32_t *__restrict__ ecells,
                                              int necell, int tile, const T *__restrict__ minv,
                                              const T *__restrict__ V, int ncols, T s1, T s2, T shift) {
  typedef LdsTile<T, NP, NW, WR, CBW, KC> C;
  typedef typename acc4<T>::type acc_t;
  typedef T vec_t __attribute__((ext_vector_type(C::VEC)));
  constexpr int CW = C::TW / CPT;                    // columns per cell
  static_assert(C::TW % CPT == 0 && CW % 16 == 0, "a 16-column fragment belongs to one cell");
  __shared__ int32_t dof_s[CPT][NP];
  __shared__ T mi_s[CPT][NP];
  __shared__ T vd_s[CPT][NP];
  __shared__ int8_t ft_s[CPT][NP];
  __shared__ __align__(16) T Ks[2][KC * C::SK];
  __shared__ __align__(16) T Xs[2][KC * C::SX];
  const int t = threadIdx.x;
  for (int sr = t; sr < CPT * NP; sr += C::NT) {
    const int sl = sr / NP, r = sr - sl * NP;
    const int e = sl < necell ? ecells[sl] : -1;
    int d = (e >= 0 && r < n_loc) ? cmap[(int64_t)e * n_loc + r] : -1;
    dof_s[sl][r] = d < 0 ? 0 : d;
    mi_s[sl][r] = d < 0 ? T(0) : minv[d];
    const int ft = d < 0 ? 0 : first_touch(r, q, e, n_el);
    ft_s[sl][r] = (int8_t)ft;
    vd_s[sl][r] = ft ? s1 * (V[d] - shift) : T(0);
  }
  __syncthreads();
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave / C::WC, wc = wave - wr * C::WC;
  const int j = lane & 15, kq = lane >> 4;
  const int col0 = tile * CW;

  // this thread's X staging slots: chunk row xr[i], tile column xc (cell
  // slot xs, column col0 + xc % CW of that cell)
  const int xc = t % C::TW;
  const int xsl = xc / CW;
  const int xrow0 = t / C::TW;                       // rows xrow0 + i * (NT / TW)
  const bool xok = col0 + (xc - xsl * CW) < ncols && xsl < necell;
  const int xcol = xok ? col0 + (xc - xsl * CW) : 0; // clamped, in bounds
  const T xscale = xok ? T(1) : T(0);
  const int32_t *xdof = dof_s[xsl];
  const T *xmi = mi_s[xsl];

  // Staging: K_ref rows of chunk c + 1 (from L2) are loaded into registers
  // while chunk c is multiplied; the gathered X rows (from HBM) XD chunks
  // ahead, in XD register sets used in turn (the loop is unrolled by XD so
  // every set is addressed statically).  Both are written to the other half
  // of the double-buffered LDS area after the chunk's MFMAs.  The X values
  // are scaled when stored, so no wait sits at the load.
  vec_t kreg[C::KPT];
  T xr0[C::XPT], xr1[C::XPT];
  constexpr int NCHT = CPLX ? 2 * C::NCH : C::NCH;   // contraction chunks
  // chunk c covers local nodes c KC - (second half ? NP : 0) + [0, KC)
  auto node0 = [&](int c) { return c * KC - ((CPLX && c >= C::NCH) ? NP : 0); };
  auto load_k = [&](int c) {
    const vec_t *Kc = reinterpret_cast<const vec_t *>(K + (int64_t)c * KC * NP);
#pragma unroll
    for (int i = 0; i < C::KPT; ++i) {
      const int v = t + C::NT * i;
      if (v < C::KV) kreg[i] = Kc[v];
    }
  };
  auto load_x = [&](int c, T(&xr)[C::XPT]) {
    const int gcol = (CPLX && c >= C::NCH) ? (xcol ^ 1) : xcol;
#pragma unroll
    for (int i = 0; i < C::XPT; ++i) {
      const int row = node0(c) + xrow0 + i * (C::NT / C::TW);
      xr[i] = X[(int64_t)xdof[row] * ldx + gcol];
    }
  };
  auto store_k = [&](int buf) {
    constexpr int RV = NP / C::VEC;                 // 16-byte vectors per K row
#pragma unroll
    for (int i = 0; i < C::KPT; ++i) {
      const int v = t + C::NT * i;
      if (v < C::KV) {
        if constexpr (C::SK == NP) {
          reinterpret_cast<vec_t *>(Ks[buf])[v] = kreg[i];
        } else {
          const int row = v / RV;
          *reinterpret_cast<vec_t *>(&Ks[buf][row * C::SK + (v - row * RV) * C::VEC]) = kreg[i];
        }
      }
    }
  };
  auto store_x = [&](int buf, int c, const T(&xr)[C::XPT]) {
    const T sgn = (CPLX && c >= C::NCH && (xcol & 1)) ? T(-1) : T(1);
#pragma unroll
    for (int i = 0; i < C::XPT; ++i) {
      const int rr = xrow0 + i * (C::NT / C::TW);
      Xs[buf][rr * C::SX + xc] = xr[i] * (xmi[node0(c) + rr] * (xscale * sgn));
    }
  };

  acc_t acc[C::RBW][CBW];
#pragma unroll
  for (int r = 0; r < C::RBW; ++r)
#pragma unroll
    for (int cb = 0; cb < CBW; ++cb) acc[r][cb] = acc_t{0, 0, 0, 0};

  load_k(0);
  load_x(0, xr0);
  store_k(0);
  store_x(0, 0, xr0);
  if (XD == 2 && NCHT > 1) load_x(1, xr1);
  __syncthreads();
  const int arow = wr * C::RBW * 16 + j;            // A fragment: K[k][arow + 16 r]
  const int bcol = wc * CBW * 16 + j;               // B fragment: Xs[k][bcol + 16 cb]
  // chunk c: the X set xl receives chunk c + XD, the set xs holds chunk c + 1
  auto chunk = [&](int c, T(&xl)[C::XPT], T(&xs)[C::XPT]) {
    const int buf = c & 1;
    if (c + 1 < NCHT) load_k(c + 1);
    if (c + XD < NCHT) load_x(c + XD, xl);
    const T *Kb = Ks[buf];
    const T *Xb = Xs[buf];
    // Software pipeline over the chunk's (step, row-block pair) stages: the
    // LDS reads of stage s + 1 (an A pair, and the B fragments when a new
    // step starts) are issued before the MFMAs of stage s, and scheduling
    // barriers keep that order, so each read has the MFMAs of one stage to
    // land in.
    constexpr int NPR = (C::RBW + 1) / 2;           // row-block pairs per step
    constexpr int NST = (KC / 4) * NPR;             // stages per chunk
    auto read_a = [&](int st, T(&a)[2]) {
      const int kk = st / NPR, rp = st - kk * NPR;
      const T *Ka = Kb + (4 * kk + kq) * C::SK + arow + 32 * rp;
      a[0] = Ka[0];
      a[1] = 2 * rp + 1 < C::RBW ? Ka[16] : T(0);
    };
    auto read_b = [&](int kk, T(&b)[CBW]) {
#pragma unroll
      for (int cb = 0; cb < CBW; ++cb) b[cb] = Xb[(4 * kk + kq) * C::SX + bcol + 16 * cb];
    };
    T a_cur[2], a_nxt[2], b_cur[CBW], b_nxt[CBW];
    read_b(0, b_cur);
    read_a(0, a_cur);
#pragma unroll
    for (int st = 0; st < NST; ++st) {
      const int kk = st / NPR, rp = st - kk * NPR;
      if (st + 1 < NST) {
        read_a(st + 1, a_nxt);
        if ((st + 1) % NPR == 0) read_b(kk + 1, b_nxt);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (2 * rp + h < C::RBW) {
#pragma unroll
          for (int cb = 0; cb < CBW; ++cb)
            acc[2 * rp + h][cb] = mfma16x4(a_cur[h], b_cur[cb], acc[2 * rp + h][cb]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      if (st + 1 < NST) {
        a_cur[0] = a_nxt[0];
        a_cur[1] = a_nxt[1];
        if ((st + 1) % NPR == 0) {
#pragma unroll
          for (int cb = 0; cb < CBW; ++cb) b_cur[cb] = b_nxt[cb];
        }
      }
    }
    if (c + 1 < NCHT) {
      store_k(buf ^ 1);
      store_x(buf ^ 1, c + 1, xs);
    }
    __syncthreads();
  };
  if constexpr (XD == 2) {
    // even c: xr0 takes chunk c + 2, xr1 holds chunk c + 1; odd c: swapped.
    // Chunk pairs per loop iteration, measured per precision and cell size
    // (128-column blocks, ms per colour launch): FP64 p = 5 and FP32 p = 6
    // the whole loop unrolled (1.031 against 1.066 with two pairs and 1.081
    // with one; 0.568 against 0.590 and 0.595); FP32 p = 5 and FP64 p = 6
    // two pairs (0.594 against 0.626 whole and 0.602 one; 1.122 against
    // 1.124 and 1.126); p = 4 two pairs (FP64 0.199 against 0.215 with one,
    // FP32 0.122 against 0.126); FP32 p = 7 one pair (0.167 against 0.181
    // with two); the complex tile whole (ms per apply of 64 complex vectors:
    // p = 5 14.10 against 14.64 with two pairs and 15.08 with one; p = 6
    // 15.72 against 19.17 and 15.85)
    constexpr bool WHOLE = CPLX || (sizeof(T) == 8 && NP == 224) || (sizeof(T) == 4 && NP == 352);
    constexpr bool ONE = sizeof(T) == 4 && NP == 512;
    constexpr int UP = ONE ? 1 : (WHOLE ? (NCHT + 1) / 2 : 2);
#pragma unroll UP
    for (int c = 0; c < NCHT; c += 2) {
      chunk(c, xr0, xr1);
      if (c + 1 < NCHT) chunk(c + 1, xr1, xr0);
    }
  } else {
#pragma unroll 1
    for (int c = 0; c < NCHT; ++c) chunk(c, xr0, xr0);
  }

  // epilogue, software-pipelined EPD - 1 fragments ahead; fragment i's 16
  // columns belong to cell slot frag_slot(i)
  constexpr int NF = C::RBW * CBW;
  auto frag_tc = [&](int i) { return wc * CBW * 16 + 16 * (i % CBW); };   // first tile column
  auto frag_slot = [&](int i) { return frag_tc(i) / CW; };
  auto frag_col = [&](int i) { return col0 + (frag_tc(i) - frag_slot(i) * CW) + j; };
  auto frag_row = [&](int i) { return (wr * C::RBW + i / CBW) * 16; };
  auto frag_ctx = [&](int i) {
    const int sl = frag_slot(i);
    return EpiCtx<T>{X, ldx, Xp, ldp, Y, ldy, dof_s[sl], mi_s[sl], vd_s[sl], ft_s[sl], n_loc, s1, s2};
  };
  auto frag_ok = [&](int i) { return frag_col(i) < ncols && frag_slot(i) < necell; };
  auto frag_load = [&](int i, EpiFrag<T> &f) {
    const int ci = frag_col(i);
    epi_load(frag_ctx(i), frag_row(i), kq, frag_ok(i) ? ci : 0, f);
  };
  EpiFrag<T> f[EPD];
#pragma unroll
  for (int i = 0; i < EPD - 1; ++i)
    if (i < NF) frag_load(i, f[i]);
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    if (i + EPD - 1 < NF) frag_load(i + EPD - 1, f[(i + EPD - 1) % EPD]);
    epi_store(frag_ctx(i), frag_row(i), kq, frag_col(i), frag_ok(i), f[i % EPD], acc[i / CBW][i % CBW]);
  }
}

// ---------------------------------------------------------------------------
// Degrees 8..12 (n_loc = 729 .. 2197): the cell matrix no longer fits one
// work-group's accumulators, so a work-group computes RT_NR = 224 output
// rows [r0, r0 + 224) of one cell for 64 columns, contracting over all local
// nodes (padded to npk, a multiple of 16).  The tile is the p = 5 eight-wave
// one (2 x 4 waves, 7 row blocks and one column block each); the cell matrix
// is stored [npk][npr] (npr = row groups x 224, zero padded), and the chunk
// count is a run-time value.  Rows at or beyond n_loc are computed on zero
// padding and not stored.
// ---------------------------------------------------------------------------
constexpr int RT_NR = 224, RT_NW = 8, RT_WC = 4, RT_RBW = 7, RT_KC = 8, RT_TW = 64;   // waves 2 x 4
constexpr int RT_NPMAX = 2240;   // p = 12: 2197 rows in ten groups of 224

template <typename T>
__global__ __launch_bounds__(64 * RT_NW) __attribute__((amdgpu_waves_per_eu(4))) void hx_rows_kernel(
    const T *__restrict__ X, int64_t ldx, const T *__restrict__ Xp, int64_t ldp, T *__restrict__ Y, int64_t ldy,
    const T *__restrict__ K, int npk, int npr, const int32_t *__restrict__ cmap, int n_loc, int q, int n_el,
    const int32_t *__restrict__ cells, const T *__restrict__ minv, const T *__restrict__ V, int ncols, int ngrp,
    int ntiles, T s1, T s2, T shift) {
  typedef typename acc4<T>::type acc_t;
  typedef T vec_t __attribute__((ext_vector_type(16 / sizeof(T))));
  constexpr int NT = 64 * RT_NW, VEC = 16 / sizeof(T);
  constexpr int SK = sizeof(T) == 4 ? RT_NR + 16 : RT_NR;      // FP32 rows padded to 16 (mod 32) words
  constexpr int SX = sizeof(T) == 4 ? RT_TW + 16 : RT_TW;
  constexpr int KV = RT_KC * RT_NR / VEC, KPT = (KV + NT - 1) / NT, XPT = RT_KC * RT_TW / NT;
  __shared__ int32_t dof_s[RT_NPMAX];
  __shared__ T mi_s[RT_NPMAX];
  __shared__ T vd_s[RT_NR];
  __shared__ int8_t ft_s[RT_NR];
  __shared__ __align__(16) T Ks[2][RT_KC * SK];
  __shared__ __align__(16) T Xs[2][RT_KC * SX];
  const int tile = blockIdx.x % ntiles;
  const int rest = blockIdx.x / ntiles;
  const int rg = rest % ngrp;
  const int e = cells[rest / ngrp];
  const int r0 = rg * RT_NR;
  const int t = threadIdx.x;
  for (int r = t; r < npr; r += NT) {
    const int d = r < n_loc ? cmap[(int64_t)e * n_loc + r] : -1;
    dof_s[r] = d < 0 ? 0 : d;
    mi_s[r] = d < 0 ? T(0) : minv[d];
  }
  for (int rr = t; rr < RT_NR; rr += NT) {
    const int r = r0 + rr;
    const int d = r < n_loc ? cmap[(int64_t)e * n_loc + r] : -1;
    const int ft = d < 0 ? 0 : first_touch(r, q, e, n_el);
    ft_s[rr] = (int8_t)ft;
    vd_s[rr] = ft ? s1 * (V[d] - shift) : T(0);
  }
  __syncthreads();
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave / RT_WC, wc = wave - wr * RT_WC;
  const int j = lane & 15, kq = lane >> 4;
  const int col0 = tile * RT_TW;
  const int xc = t % RT_TW, xrow0 = t / RT_TW;
  const bool xok = col0 + xc < ncols;
  const int xcol = xok ? col0 + xc : 0;
  const T xscale = xok ? T(1) : T(0);
  const int nch = npk / RT_KC;
  vec_t kreg[KPT];
  T xreg[XPT];
  auto load_chunk = [&](int c) {
    const T *Kc = K + (int64_t)c * RT_KC * npr + r0;
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const int v = t + NT * i;
      if (v < KV) {
        const int row = v / (RT_NR / VEC), cv = v - row * (RT_NR / VEC);
        kreg[i] = *reinterpret_cast<const vec_t *>(Kc + (int64_t)row * npr + cv * VEC);
      }
    }
#pragma unroll
    for (int i = 0; i < XPT; ++i) {
      const int row = c * RT_KC + xrow0 + i * (NT / RT_TW);
      xreg[i] = X[(int64_t)dof_s[row] * ldx + xcol];
    }
  };
  auto store_chunk = [&](int buf, int c) {
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const int v = t + NT * i;
      if (v < KV) {
        const int row = v / (RT_NR / VEC), cv = v - row * (RT_NR / VEC);
        *reinterpret_cast<vec_t *>(&Ks[buf][row * SK + cv * VEC]) = kreg[i];
      }
    }
#pragma unroll
    for (int i = 0; i < XPT; ++i) {
      const int rr = xrow0 + i * (NT / RT_TW);
      Xs[buf][rr * SX + xc] = xreg[i] * (mi_s[c * RT_KC + rr] * xscale);
    }
  };
  acc_t acc[RT_RBW];
#pragma unroll
  for (int r = 0; r < RT_RBW; ++r) acc[r] = acc_t{0, 0, 0, 0};
  load_chunk(0);
  store_chunk(0, 0);
  __syncthreads();
  const int arow = wr * RT_RBW * 16 + j;
  const int bcol = wc * 16 + j;
#pragma unroll 1
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) load_chunk(c + 1);
    const T *Kb = Ks[buf];
    const T *Xb = Xs[buf];
#pragma unroll
    for (int kk = 0; kk < RT_KC / 4; ++kk) {
      const T b = Xb[(4 * kk + kq) * SX + bcol];
#pragma unroll
      for (int r = 0; r < RT_RBW; ++r) acc[r] = mfma16x4(Kb[(4 * kk + kq) * SK + arow + 16 * r], b, acc[r]);
    }
    if (c + 1 < nch) store_chunk(buf ^ 1, c + 1);
    __syncthreads();
  }
  // epilogue on the group's rows (row indices local to the group)
  const EpiCtx<T> ec{X, ldx, Xp, ldp, Y, ldy, dof_s + r0, mi_s + r0, vd_s, ft_s, n_loc - r0, s1, s2};
  const int ci = col0 + bcol;
  const bool cok = ci < ncols;
#pragma unroll
  for (int r = 0; r < RT_RBW; ++r) {
    EpiFrag<T> f;
    const int row0 = (wr * RT_RBW + r) * 16;
    epi_load(ec, row0, kq, cok ? ci : 0, f);
    epi_store(ec, row0, kq, ci, cok, f, acc[r]);
  }
}

template <typename T>
int hx_rows_launch(const HxArgs<T> &a, int npr, int color_begin, int color_end, hipStream_t s) {
  const int ncell = color_end - color_begin;
  const int ntiles = (a.ncols + RT_TW - 1) / RT_TW;
  const int ngrp = npr / RT_NR;
  if (ncell <= 0 || ntiles <= 0) return 0;
  if (npr % RT_NR || npr > RT_NPMAX || a.np % 16 || a.np > npr) return -1;
  if ((int64_t)ncell * ngrp * ntiles > INT32_MAX) return -1;
  hipLaunchKernelGGL((hx_rows_kernel<T>), dim3((unsigned)(ncell * ngrp * ntiles)), dim3(64 * RT_NW), 0, s, a.X,
                     a.ldx, a.Xp, a.ldp, a.Y, a.ldy, a.K, a.np, npr, a.cmap, a.n_loc, a.q, a.n_el,
                     a.cells + color_begin, a.minv, a.V, a.ncols, ngrp, ntiles, a.s1, a.s2, a.shift);
  return 0;
}
template int hx_rows_launch<double>(const HxArgs<double> &, int, int, int, hipStream_t);
template int hx_rows_launch<float>(const HxArgs<float> &, int, int, int, hipStream_t);

int hx_rows_padded(int n_loc) { return (n_loc + RT_NR - 1) / RT_NR * RT_NR; }

// ---------------------------------------------------------------------------
// BF16 cell products (FP32 state, FP32 accumulation): v_mfma_f32_16x16x32_bf16.
// The cell's gathered, M^-1/2-scaled X rows (64 columns) are converted to BF16
// (round to nearest even) and staged in LDS transposed, [column][local node],
// so a B fragment (8 consecutive local nodes of one column) is one 16-byte LDS
// read.  SPLIT: X = hi + lo and K = hi + lo in BF16, three products
// hi*hi + hi*lo + lo*hi accumulated in FP32.  NPB: n_loc rounded up to 32.
// ---------------------------------------------------------------------------
// EPD: epilogue fragments in flight (3 measured no faster than 2).
// CBW: 16-column blocks per wave, so a work-group covers TWB = 32 CBW columns
// (two blocks: every K fragment feeds two MFMAs; one block: half the LDS per
// work-group, so more work-groups share a CU and overlap their gathers and
// epilogues).
// One kernel for both launch forms, so that the tile body sits directly in
// the kernel (the same body inlined from a device function gets a register
// allocation of up to 296 per lane at p = 6 and one wave per SIMD):
//  * single problem: work-group = (cell of the colour list, column tile),
//    operands from the kernel arguments;
//  * BATCH: work item (problem, cell position in the problem's colour-sorted
//    list, column tile) from a device list, operands from the problem's
//    descriptor, coefficients from its table (s1, s2, shift per step).
// One work-group = one cell e x TWB columns from tile * TWB.
template <int NPB, bool SPLIT, int CBW, bool BATCH>
__global__ __launch_bounds__(256) void hx_cells_bf16_kernel(
    const float *__restrict__ X_, int64_t ldx_, const float *__restrict__ Xp_, int64_t ldp_, float *__restrict__ Y_,
    int64_t ldy_, const __bf16 *__restrict__ Kh_, const __bf16 *__restrict__ Kl_, const int32_t *__restrict__ cmap_,
    int n_loc_, int q_, int n_el_, const int32_t *__restrict__ cells_, const float *__restrict__ minv_,
    const float *__restrict__ V_, int ncols_, int ntiles, float s1_, float s2_, float shift_,
    const BatchProblemBf16 *__restrict__ probs, const int4 *__restrict__ work, int step, int cur, int prev, int out) {
  const float *X, *Xp, *minv, *V;
  float *Y;
  int64_t ldx, ldp, ldy;
  const __bf16 *Kh, *Kl;
  const int32_t *cmap;
  int n_loc, q, n_el, ncols, e, tile;
  float s1, s2, shift;
  if constexpr (BATCH) {
    const int4 w = work[blockIdx.x];
    const BatchProblemBf16 &P = probs[w.x];
    const float *coef = P.coef + 3 * step;
    X = P.buf[cur];
    ldx = P.ld[cur];
    Xp = prev >= 0 ? P.buf[prev] : nullptr;
    ldp = prev >= 0 ? P.ld[prev] : 0;
    Y = P.buf[out];
    ldy = P.ld[out];
    Kh = P.Kh;
    Kl = P.Kl;
    cmap = P.cmap;
    n_loc = P.n_loc;
    q = P.q;
    n_el = P.n_el;
    minv = P.minv;
    V = P.V;
    ncols = P.ncols;
    e = P.cells[w.y];
    tile = w.z;
    s1 = coef[0];
    s2 = coef[1];
    shift = coef[2];
  } else {
    X = X_;
    ldx = ldx_;
    Xp = Xp_;
    ldp = ldp_;
    Y = Y_;
    ldy = ldy_;
    Kh = Kh_;
    Kl = Kl_;
    cmap = cmap_;
    n_loc = n_loc_;
    q = q_;
    n_el = n_el_;
    minv = minv_;
    V = V_;
    ncols = ncols_;
    const int cell_slot = blockIdx.x / ntiles;
    tile = blockIdx.x - cell_slot * ntiles;
    e = cells_[cell_slot];
    s1 = s1_;
    s2 = s2_;
    shift = shift_;
  }
  constexpr int EPD = 2;                   // epilogue fragments in flight (3 measured no faster)

  constexpr int RB = NPB / 16;
  constexpr int LDX = NPB + 8;            // row of the transposed tile, 16-byte aligned
  constexpr int NPART = SPLIT ? 2 : 1;
  __shared__ int32_t dof_s[NPB];
  __shared__ float mi_s[NPB];
  __shared__ float vd_s[NPB];
  __shared__ int8_t ft_s[NPB];
  constexpr int TWB = 32 * CBW;          // columns per work-group
  const int col0 = tile * TWB;
  constexpr int NG4 = TWB / 4;            // groups of four columns
  __shared__ __attribute__((aligned(16))) __bf16 xs[NPART][TWB * LDX];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int r = threadIdx.x; r < NPB; r += blockDim.x) {
    int d = r < n_loc ? cmap[(int64_t)e * n_loc + r] : -1;
    dof_s[r] = d < 0 ? 0 : d;
    mi_s[r] = d < 0 ? 0.f : minv[d];
    const int ft = d < 0 ? 0 : first_touch(r, q, e, n_el);
    ft_s[r] = (int8_t)ft;
    vd_s[r] = ft ? s1 * (V[d] - shift) : 0.f;
  }
  __syncthreads();
  // stage: 4 consecutive columns per thread per row (16-byte global loads when
  // aligned), SU rows per thread per round with every load issued first
  const bool vec_ok = ((ldx & 3) == 0) && ((col0 & 3) == 0) && ((((uintptr_t)X) & 15) == 0);
  constexpr int SU = 8;   // (all 22 rows at once measured no faster)
  for (int base = threadIdx.x; base < NPB * NG4; base += SU * 256) {
    float v[SU][4];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int idx = base + u * 256;
      v[u][0] = v[u][1] = v[u][2] = v[u][3] = 0.f;
      if (idx < NPB * NG4) {
        const int r = idx / NG4, c4 = (idx % NG4) * 4;
        const float *src = X + (int64_t)dof_s[r] * ldx + col0 + c4;
        if (vec_ok && col0 + c4 + 3 < ncols) {
          const float4 t = *reinterpret_cast<const float4 *>(src);
          v[u][0] = t.x; v[u][1] = t.y; v[u][2] = t.z; v[u][3] = t.w;
        } else {
#pragma unroll
          for (int w = 0; w < 4; ++w) v[u][w] = (col0 + c4 + w < ncols) ? src[w] : 0.f;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int idx = base + u * 256;
      if (idx < NPB * NG4) {
        const int r = idx / NG4, c4 = (idx % NG4) * 4;
        const float w = mi_s[r];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float x = v[u][t] * w;
          const __bf16 h = (__bf16)x;
          xs[0][(c4 + t) * LDX + r] = h;
          if (SPLIT) xs[NPART - 1][(c4 + t) * LDX + r] = (__bf16)(x - (float)h);
        }
      }
    }
  }
  __syncthreads();
  // waves in a 2 x 2 grid: wave (wr, wc) owns row blocks [wr*RBW, (wr+1)*RBW)
  // and the two 16-column blocks of columns [32 wc, 32 wc + 32), so every K
  // fragment loaded from L2 feeds two MFMAs and each wave reads half of K.
  constexpr int RBW = RB / 2;
  const int wr = wave >> 1, wc = wave & 1;
  const int j = lane & 15, kq = lane >> 4;
  v4f acc[RBW][CBW];
#pragma unroll
  for (int r = 0; r < RBW; ++r)
#pragma unroll
    for (int cb = 0; cb < CBW; ++cb) acc[r][cb] = v4f{0, 0, 0, 0};
  typedef __attribute__((ext_vector_type(4))) int v4i;
  const __bf16 *Kh_w = Kh + (int64_t)(wr * RBW * 16 + j) * NPB + 8 * kq;   // A[i][k..k+7] = K[i][k..k+7]
  const __bf16 *Kl_w = SPLIT ? Kl + (int64_t)(wr * RBW * 16 + j) * NPB + 8 * kq : nullptr;
  auto load_a = [&](const __bf16 *Kp, int k, int r) {
    return __builtin_bit_cast(v8bf, *reinterpret_cast<const v4i *>(Kp + (int64_t)r * 16 * NPB + k));
  };
  // hi fragments one k-step ahead in ping-pong registers; split, the lo
  // fragments too from 352 padded rows up (measured at p = 6: 0.62 against
  // 0.75 ms per colour launch; at p = 5, where the two 64-column tiles
  // already limit a CU to two work-groups, loading them in the loop is 3 %
  // faster)
  constexpr bool PRE_LO = SPLIT && NPB >= 352;
  constexpr int RLO = PRE_LO ? RBW : 1;
  v8bf ah[2][RBW], al[2][RLO];
#pragma unroll
  for (int r = 0; r < RBW; ++r) ah[0][r] = load_a(Kh_w, 0, r);
  if constexpr (PRE_LO) {
#pragma unroll
    for (int r = 0; r < RBW; ++r) al[0][r] = load_a(Kl_w, 0, r);
  }
  if constexpr (!SPLIT && NPB == 224) {
    // p = 5: the seven k-steps fully unrolled (same ping-pong, no loop):
    // 0.435 against 0.465 ms per colour launch at 32^3 cells, 128 columns; a
    // three-deep ring measured the same, and at p = 6 full unrolling costs a
    // work-group per CU (0.436 against 0.362 ms)
    constexpr int NKS = NPB / 32;
#pragma unroll
    for (int t = 0; t < NKS; ++t) {
      if (t + 1 < NKS) {
#pragma unroll
        for (int r = 0; r < RBW; ++r) ah[(t + 1) & 1][r] = load_a(Kh_w, 32 * (t + 1), r);
      }
      v8bf bh[CBW];
#pragma unroll
      for (int cb = 0; cb < CBW; ++cb) {
        const int lc = wc * 16 * CBW + cb * 16 + j;
        bh[cb] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4i *>(&xs[0][lc * LDX + 32 * t + 8 * kq]));
      }
#pragma unroll
      for (int r = 0; r < RBW; ++r)
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb) acc[r][cb] = mfma16x32bf(ah[t & 1][r], bh[cb], acc[r][cb]);
    }
  } else
#pragma unroll 1
  for (int k = 0; k < NPB; k += 64) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int kk = k + 32 * u;
      if (kk >= NPB) break;                       // NPB is a multiple of 32
      const int kn = kk + 32 < NPB ? kk + 32 : kk;
#pragma unroll
      for (int r = 0; r < RBW; ++r) ah[u ^ 1][r] = load_a(Kh_w, kn, r);
      if constexpr (PRE_LO) {
#pragma unroll
        for (int r = 0; r < RBW; ++r) al[u ^ 1][r] = load_a(Kl_w, kn, r);
      }
      v8bf bh[CBW], bl[CBW];
#pragma unroll
      for (int cb = 0; cb < CBW; ++cb) {
        const int lc = wc * 16 * CBW + cb * 16 + j;
        bh[cb] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4i *>(&xs[0][lc * LDX + kk + 8 * kq]));
        if (SPLIT) bl[cb] = __builtin_bit_cast(v8bf, *reinterpret_cast<const v4i *>(&xs[NPART - 1][lc * LDX + kk + 8 * kq]));
      }
#pragma unroll
      for (int r = 0; r < RBW; ++r) {
#pragma unroll
        for (int cb = 0; cb < CBW; ++cb) acc[r][cb] = mfma16x32bf(ah[u][r], bh[cb], acc[r][cb]);
        if constexpr (SPLIT) {
          const v8bf alr = PRE_LO ? al[u][r % RLO] : load_a(Kl_w, kk, r);
#pragma unroll
          for (int cb = 0; cb < CBW; ++cb) {
            acc[r][cb] = mfma16x32bf(ah[u][r], bl[cb], acc[r][cb]);
            acc[r][cb] = mfma16x32bf(alr, bh[cb], acc[r][cb]);
          }
        }
      }
    }
  }

  // epilogue, software-pipelined EPD - 1 fragments ahead
  const EpiCtx<float> ec{X, ldx, Xp, ldp, Y, ldy, dof_s, mi_s, vd_s, ft_s, n_loc, s1, s2};
  constexpr int NF = RBW * CBW;
  auto frag_col = [&](int i) { return col0 + wc * 16 * CBW + 16 * (i % CBW) + j; };
  auto frag_row = [&](int i) { return (wr * RBW + i / CBW) * 16; };
  auto frag_load = [&](int i, EpiFrag<float> &f) {
    const int ci = frag_col(i);
    epi_load(ec, frag_row(i), kq, ci < ncols ? ci : ncols - 1, f);
  };
  EpiFrag<float> f[EPD];
#pragma unroll
  for (int i = 0; i < EPD - 1; ++i)
    if (i < NF) frag_load(i, f[i]);
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    if (i + EPD - 1 < NF) frag_load(i + EPD - 1, f[(i + EPD - 1) % EPD]);
    const int ci = frag_col(i);
    epi_store(ec, frag_row(i), kq, ci, ci < ncols, f[i % EPD], acc[i / CBW][i % CBW]);
  }
}

template <int NPB, bool SPLIT, int CBW>
static void launch_bf16(const HxBf16Args &a, int color_begin, int color_end, hipStream_t s) {
  constexpr int TWB = 32 * CBW;
  int ntiles = (a.ncols + TWB - 1) / TWB;
  int ncell = color_end - color_begin;
  if (ncell <= 0 || ntiles <= 0) return;
  hipLaunchKernelGGL((hx_cells_bf16_kernel<NPB, SPLIT, CBW, false>), dim3((unsigned)(ncell * ntiles)), dim3(256), 0, s,
                     a.X, a.ldx, a.Xp, a.ldp, a.Y, a.ldy, a.Kh, a.Kl, a.cmap, a.n_loc, a.q, a.n_el,
                     a.cells + color_begin, a.minv, a.V, a.ncols, ntiles, a.s1, a.s2, a.shift, nullptr, nullptr, 0, 0,
                     0, 0);
}

template <bool SPLIT, int CBW>
static int dispatch_bf16_w(const HxBf16Args &a, int cb, int ce, hipStream_t s) {
  switch (a.npb) {
    case 32: launch_bf16<32, SPLIT, CBW>(a, cb, ce, s); break;
    case 64: launch_bf16<64, SPLIT, CBW>(a, cb, ce, s); break;
    case 128: launch_bf16<128, SPLIT, CBW>(a, cb, ce, s); break;
    case 224: launch_bf16<224, SPLIT, CBW>(a, cb, ce, s); break;
    case 352: launch_bf16<352, SPLIT, CBW>(a, cb, ce, s); break;
    case 512: launch_bf16<512, SPLIT, CBW>(a, cb, ce, s); break;
    default: return -1;
  }
  return 0;
}

template <bool SPLIT>
static int dispatch_bf16(const HxBf16Args &a, int cb, int ce, hipStream_t s) {
  return a.cbw == 1 ? dispatch_bf16_w<SPLIT, 1>(a, cb, ce, s) : dispatch_bf16_w<SPLIT, 2>(a, cb, ce, s);
}

int hx_cells_bf16_launch(const HxBf16Args &a, int color_begin, int color_end, hipStream_t s) {
  return a.split ? dispatch_bf16<true>(a, color_begin, color_end, s) : dispatch_bf16<false>(a, color_begin, color_end, s);
}

template <bool SPLIT>
static int bf16_batch_dispatch(int npb, const BatchProblemBf16 *probs, const int4 *work, int nwork, int step, int cur,
                               int prev, int out, hipStream_t s) {
  const dim3 g((unsigned)nwork), b(256);
  switch (npb) {
#define CHFSI_BF16_BATCH(NPB)                                                                                   \
  case NPB:                                                                                                     \
    hipLaunchKernelGGL((hx_cells_bf16_kernel<NPB, SPLIT, 2, true>), g, b, 0, s, nullptr, 0, nullptr, 0, nullptr, 0,   \
                       nullptr, nullptr, nullptr, 0, 0, 0, nullptr, nullptr, nullptr, 0, 1, 0.f, 0.f, 0.f, probs,     \
                       work, step, cur, prev, out);                                                             \
    return 0;
    CHFSI_BF16_BATCH(32) CHFSI_BF16_BATCH(64) CHFSI_BF16_BATCH(128) CHFSI_BF16_BATCH(224) CHFSI_BF16_BATCH(352)
    CHFSI_BF16_BATCH(512)
#undef CHFSI_BF16_BATCH
    default: return -1;
  }
}

int hx_cells_bf16_batch_launch(int npb, int split, const BatchProblemBf16 *probs, const int4 *work, int nwork,
                               int step, int cur, int prev, int out, hipStream_t s) {
  if (nwork <= 0) return 0;
  return split ? bf16_batch_dispatch<true>(npb, probs, work, nwork, step, cur, prev, out, s)
               : bf16_batch_dispatch<false>(npb, probs, work, nwork, step, cur, prev, out, s);
}

// Tile configurations per padded cell size: waves per work-group, the split
// of the row blocks over waves, column blocks per wave, contraction chunk.
//  * variant 0: four waves, 2 x 2 grid, two column blocks per wave (the A
//    fragment of every LDS read feeds two MFMAs); p = 7 splits its 32 row
//    blocks over four waves;
//  * variant 1: eight waves, 2 x 4 grid, one column block per wave: half the
//    accumulators, so four waves per SIMD instead of two.  Only where the
//    accumulators fit 128 registers (FP64 up to p = 5, FP32 up to p = 7);
//    elsewhere variant 1 is variant 0.
// The built-in choice (variant -1) is variant 1 for FP64 p = 5 and FP32
// p = 6 (measured faster there: 1.08 against 1.30 ms and 0.59 against 0.66
// ms per colour launch of 128 columns) and variant 0 otherwise; the
// autotuner times both.
template <typename T, int NP, int V>
struct TileCfg {
  static constexpr bool w8 = V == 1 && NP >= 32 && (sizeof(T) == 8 ? NP <= 224 : NP <= 512);
  static constexpr int NW = w8 ? 8 : 4;
  static constexpr int WR = NP == 16 ? 1 : ((NP == 512 && !w8) ? 4 : 2);
  static constexpr int CBW = (NP == 16 || w8) ? 1 : 2;
  static constexpr int KC = 8;
  static constexpr int EPD = 2;   // epilogue fragments in flight (3 measured no faster)
  typedef LdsTile<T, NP, NW, WR, CBW, KC> L;
  // eight-wave tiles must keep four waves per SIMD (two work-groups per CU)
  static constexpr int WAVES = NW == 8 ? 4 : 1;
};

template <typename T>
static int default_variant(int np) {
  // measured at 32^3 cells p = 5 and 24^3 cells p = 6, 128-column blocks
  if (sizeof(T) == 8) return np == 224 ? 1 : 0;
  return np == 352 ? 1 : 0;
}

#define CHFSI_CELL_TILE(T, NP, V, CPT, ...)                                                                  \
  cell_tile<T, NP, TileCfg<T, NP, V>::NW, TileCfg<T, NP, V>::WR, TileCfg<T, NP, V>::CBW, TileCfg<T, NP, V>::KC, \
            TileCfg<T, NP, V>::EPD, false, CPT>(__VA_ARGS__)

// Work-group = (group of CPT cells of the colour, column tile).
template <typename T, int NP, int V, int CPT>
__global__ __launch_bounds__((64 * TileCfg<T, NP, V>::NW))
__attribute__((amdgpu_waves_per_eu(TileCfg<T, NP, V>::WAVES))) void hx_cells_kernel(
    const T *__restrict__ X, int64_t ldx, const T *__restrict__ Xp, int64_t ldp, T *__restrict__ Y, int64_t ldy,
    const T *__restrict__ K, const int32_t *__restrict__ cmap, int n_loc, int q, int n_el,
    const int32_t *__restrict__ cells, int ncell, const T *__restrict__ minv, const T *__restrict__ V_, int ncols,
    int ntiles, T s1, T s2, T shift) {
  const int grp = blockIdx.x / ntiles;
  const int tile = blockIdx.x - grp * ntiles;
  const int first = grp * CPT;
  const int cnt = ncell - first < CPT ? ncell - first : CPT;
  CHFSI_CELL_TILE(T, NP, V, CPT, X, ldx, Xp, ldp, Y, ldy, K, cmap, n_loc, q, n_el, cells + first, cnt, tile, minv,
                  V_, ncols, s1, s2, shift);
}

// Batched: work item = (problem, first cell in the problem's colour-sorted
// cell list, column tile, cell count); the step's buffer roles (input,
// previous, output) are the same for every problem, its coefficients come
// from the problem's table (s1, s2, shift per step).
template <typename T, int NP, int V, int CPT>
__global__ __launch_bounds__((64 * TileCfg<T, NP, V>::NW))
__attribute__((amdgpu_waves_per_eu(TileCfg<T, NP, V>::WAVES))) void hx_cells_batch_kernel(
    const BatchProblem<T> *__restrict__ probs, const int4 *__restrict__ work, int step, int cur, int prev, int out) {
  const int4 w = work[blockIdx.x];
  const BatchProblem<T> &P = probs[w.x];
  const T *coef = P.coef + 3 * step;
  CHFSI_CELL_TILE(T, NP, V, CPT, P.buf[cur], P.ld[cur], prev >= 0 ? P.buf[prev] : nullptr,
                  prev >= 0 ? P.ld[prev] : 0, P.buf[out], P.ld[out], P.K, P.cmap, P.n_loc, P.q, P.n_el,
                  P.cells + w.y, w.w, w.z, P.minv, P.V, P.ncols, coef[0], coef[1], coef[2]);
}

// Complex Bloch operator on a periodic mesh (FP64): the same tile with the
// doubled contraction.
// The recursion coefficients are real, so a Chebyshev step on complex
// blocks is the same element-wise epilogue on the interleaved values.
template <int NP, int V>
__global__ __launch_bounds__((64 * TileCfg<double, NP, V>::NW))
__attribute__((amdgpu_waves_per_eu(TileCfg<double, NP, V>::WAVES))) void hx_cells_cplx_kernel(
    const double *__restrict__ X, int64_t ldx, const double *__restrict__ Xp, int64_t ldp, double *__restrict__ Y,
    int64_t ldy, const double *__restrict__ K, const int32_t *__restrict__ cmap, int n_loc, int q, int n_el,
    const int32_t *__restrict__ cells, const double *__restrict__ minv, const double *__restrict__ V_, int ncols,
    int ntiles, double s1, double s2, double shift) {
  typedef TileCfg<double, NP, V> CF;
  const int cell_slot = blockIdx.x / ntiles;
  const int tile = blockIdx.x - cell_slot * ntiles;
  cell_tile<double, NP, CF::NW, CF::WR, CF::CBW, CF::KC, CF::EPD, true>(
      X, ldx, Xp, ldp, Y, ldy, K, cmap, n_loc, q, n_el, cells + cell_slot, 1, tile, minv, V_, ncols, s1, s2, shift);
}

// A group of k-points on one mesh: work item (k, cell, column tile); k's
// block, cell operator and |k|^2/2 shift sit at fixed strides.
template <int NP, int V>
__global__ __launch_bounds__((64 * TileCfg<double, NP, V>::NW))
__attribute__((amdgpu_waves_per_eu(TileCfg<double, NP, V>::WAVES))) void hx_cells_cplx_kpts_kernel(
    const double *__restrict__ X, int64_t ldx, int64_t xstride, double *__restrict__ Y, int64_t ldy,
    int64_t ystride, const double *__restrict__ K, int64_t kstride, const double *__restrict__ shifts,
    const int32_t *__restrict__ cmap, int n_loc, int q, int n_el, const int32_t *__restrict__ cells,
    const double *__restrict__ minv, const double *__restrict__ V_, int ncols, int ntiles, int ncell) {
  typedef TileCfg<double, NP, V> CF;
  const int per_k = ncell * ntiles;
  const int kk = blockIdx.x / per_k;
  const int rest = blockIdx.x - kk * per_k;
  const int cell_slot = rest / ntiles;
  const int tile = rest - cell_slot * ntiles;
  cell_tile<double, NP, CF::NW, CF::WR, CF::CBW, CF::KC, CF::EPD, true>(
      X + kk * xstride, ldx, nullptr, 0, Y + kk * ystride, ldy, K + kk * kstride, cmap, n_loc, q, n_el,
      cells + cell_slot, 1, tile, minv, V_, ncols, 1.0, 0.0, shifts[kk]);
}
#undef CHFSI_CELL_TILE

template <typename T, int NP, int V, int CPT>
static void launch_cells(const HxArgs<T> &a, int color_begin, int color_end, hipStream_t s) {
  constexpr int CW = TileCfg<T, NP, V>::L::TW / CPT;
  const int ntiles = (a.ncols + CW - 1) / CW;
  const int ncell = color_end - color_begin;
  if (ncell <= 0 || ntiles <= 0) return;
  const int ngrp = (ncell + CPT - 1) / CPT;
  hipLaunchKernelGGL((hx_cells_kernel<T, NP, V, CPT>), dim3((unsigned)(ngrp * ntiles)),
                     dim3(64 * TileCfg<T, NP, V>::NW), 0, s, a.X, a.ldx, a.Xp, a.ldp, a.Y, a.ldy, a.K, a.cmap,
                     a.n_loc, a.q, a.n_el, a.cells + color_begin, ncell, a.minv, a.V, a.ncols, ntiles, a.s1, a.s2,
                     a.shift);
}

template <int NP, int V>
static void launch_cells_cplx(const HxArgs<double> &a, int color_begin, int color_end, hipStream_t s) {
  constexpr int TW = TileCfg<double, NP, V>::L::TW;
  static_assert(TW % 2 == 0, "complex column pairs must not straddle a tile");
  const int ntiles = (a.ncols + TW - 1) / TW;
  const int ncell = color_end - color_begin;
  if (ncell <= 0 || ntiles <= 0) return;
  hipLaunchKernelGGL((hx_cells_cplx_kernel<NP, V>), dim3((unsigned)(ncell * ntiles)),
                     dim3(64 * TileCfg<double, NP, V>::NW), 0, s, a.X, a.ldx, a.Xp, a.ldp, a.Y, a.ldy, a.K, a.cmap,
                     a.n_loc, a.q, a.n_el, a.cells + color_begin, a.minv, a.V, a.ncols, ntiles, a.s1, a.s2, a.shift);
}

template <int NP, int V>
static void launch_cells_cplx_kpts(const HxArgs<double> &a, const CplxKpts &g, int color_begin, int color_end,
                                   hipStream_t s) {
  constexpr int TW = TileCfg<double, NP, V>::L::TW;
  const int ntiles = (a.ncols + TW - 1) / TW;
  const int ncell = color_end - color_begin;
  if (ncell <= 0 || ntiles <= 0 || g.nk <= 0) return;
  hipLaunchKernelGGL((hx_cells_cplx_kpts_kernel<NP, V>), dim3((unsigned)(g.nk * ncell * ntiles)),
                     dim3(64 * TileCfg<double, NP, V>::NW), 0, s, a.X, a.ldx, g.xstride, a.Y, a.ldy, g.ystride, a.K,
                     g.kstride, g.shifts, a.cmap, a.n_loc, a.q, a.n_el, a.cells + color_begin, a.minv, a.V, a.ncols,
                     ntiles, ncell);
}

template <typename T, int NP, int V, int CPT>
static void launch_batch(const BatchProblem<T> *probs, const int4 *work, int nwork, int step, int cur, int prev,
                         int out, hipStream_t s) {
  if (nwork <= 0) return;
  hipLaunchKernelGGL((hx_cells_batch_kernel<T, NP, V, CPT>), dim3((unsigned)nwork),
                     dim3(64 * TileCfg<T, NP, V>::NW), 0, s, probs, work, step, cur, prev, out);
}

// Calls f.template run<NP, V, CPT>() for a supported padded cell size, tile
// variant (-1: the built-in choice) and cells per tile (1, 2 or 4, with at
// least 16 columns per cell); -1 otherwise.
template <typename T, int NP, int V, typename F>
static int with_cpt(int cpt, F &f) {
  constexpr int TW = TileCfg<T, NP, V>::L::TW;
  if (cpt == 1) {
    f.template run<NP, V, 1>();
    return 0;
  }
  // (four-cell-per-tile and two-cell tiles above p = 6 would need more
  // registers or LDS than their tiles have to spare)
  if constexpr (TW >= 32 && NP <= 352)
    if (cpt == 2) {
      f.template run<NP, V, 2>();
      return 0;
    }
  if constexpr (TW >= 64 && NP <= 352)
    if (cpt == 4) {
      f.template run<NP, V, 4>();
      return 0;
    }
  return -1;
}

template <typename T, typename F>
static int with_cfg(int np, int variant, int cpt, F &&f) {
  if (variant < 0) variant = default_variant<T>(np);
  if (variant > 1) return -1;
#define CHFSI_NP_CASE(N) \
  case N:                \
    return variant == 0 ? with_cpt<T, N, 0>(cpt, f) : with_cpt<T, N, 1>(cpt, f);
  switch (np) {
    CHFSI_NP_CASE(16)    // p = 1
    CHFSI_NP_CASE(32)    // p = 2
    CHFSI_NP_CASE(64)    // p = 3
    CHFSI_NP_CASE(128)   // p = 4
    CHFSI_NP_CASE(224)   // p = 5
    CHFSI_NP_CASE(352)   // p = 6
    CHFSI_NP_CASE(512)   // p = 7
    default: return -1;
  }
#undef CHFSI_NP_CASE
}

template <typename T>
struct TileWidthOp {
  int tw = 0;
  template <int NP, int V, int CPT> void run() { tw = TileCfg<T, NP, V>::L::TW / CPT; }
};
template <typename T>
int hx_tile_width(int np, int variant, int cpt) {
  TileWidthOp<T> op;
  return with_cfg<T>(np, variant, cpt, op) == 0 ? op.tw : -1;
}
template int hx_tile_width<double>(int, int, int);
template int hx_tile_width<float>(int, int, int);

template <typename T>
struct LaunchCellsOp {
  const HxArgs<T> &a;
  int cb, ce;
  hipStream_t s;
  template <int NP, int V, int CPT> void run() { launch_cells<T, NP, V, CPT>(a, cb, ce, s); }
};
template <typename T>
int hx_cells_launch(const HxArgs<T> &a, int color_begin, int color_end, hipStream_t s) {
  LaunchCellsOp<T> op{a, color_begin, color_end, s};
  return with_cfg<T>(a.np, a.variant, a.cpt, op);
}
template int hx_cells_launch<double>(const HxArgs<double> &, int, int, hipStream_t);
template int hx_cells_launch<float>(const HxArgs<float> &, int, int, hipStream_t);

struct LaunchCellsCplxOp {
  const HxArgs<double> &a;
  int cb, ce;
  hipStream_t s;
  template <int NP, int V, int CPT> void run() {
    if constexpr (CPT == 1) launch_cells_cplx<NP, V>(a, cb, ce, s);
  }
};
int hx_cells_cplx_launch(const HxArgs<double> &a, int color_begin, int color_end, hipStream_t s) {
  if (a.ncols % 2) return -1;
  LaunchCellsCplxOp op{a, color_begin, color_end, s};
  return with_cfg<double>(a.np, a.variant, 1, op);
}

struct LaunchCellsCplxKptsOp {
  const HxArgs<double> &a;
  const CplxKpts &g;
  int cb, ce;
  hipStream_t s;
  template <int NP, int V, int CPT> void run() {
    if constexpr (CPT == 1) launch_cells_cplx_kpts<NP, V>(a, g, cb, ce, s);
  }
};
int hx_cells_cplx_kpts_launch(const HxArgs<double> &a, const CplxKpts &g, int color_begin, int color_end,
                              hipStream_t s) {
  if (a.ncols % 2) return -1;
  if ((int64_t)g.nk * (color_end - color_begin) * ((a.ncols + 31) / 32) > INT32_MAX) return -1;   // TW >= 32
  LaunchCellsCplxKptsOp op{a, g, color_begin, color_end, s};
  return with_cfg<double>(a.np, a.variant, 1, op);
}

template <typename T>
struct LaunchBatchOp {
  const BatchProblem<T> *probs;
  const int4 *work;
  int nwork, step, cur, prev, out;
  hipStream_t s;
  template <int NP, int V, int CPT> void run() {
    launch_batch<T, NP, V, CPT>(probs, work, nwork, step, cur, prev, out, s);
  }
};
template <typename T>
int hx_cells_batch_launch(int np, int variant, int cpt, const BatchProblem<T> *probs, const int4 *work, int nwork,
                          int step, int cur, int prev, int out, hipStream_t s) {
  LaunchBatchOp<T> op{probs, work, nwork, step, cur, prev, out, s};
  return with_cfg<T>(np, variant, cpt, op);
}
template int hx_cells_batch_launch<double>(int, int, int, const BatchProblem<double> *, const int4 *, int, int, int,
                                           int, int, hipStream_t);
template int hx_cells_batch_launch<float>(int, int, int, const BatchProblem<float> *, const int4 *, int, int, int,
                                          int, int, hipStream_t);
// ---------------------------------------------------------------------------
// Precision conversion and column-block copies (strided, DoF-major)
// ---------------------------------------------------------------------------
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void copy_cols_kernel(const Tin *__restrict__ in, int64_t ldi,
                                                        Tout *__restrict__ out, int64_t ldo, int64_t nrows,
                                                        int ncols) {
  const int64_t total = nrows * (int64_t)ncols;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = t / ncols;
    int j = (int)(t - i * ncols);
    out[i * ldo + j] = (Tout)in[i * ldi + j];
  }
}

template <typename Tin, typename Tout>
void copy_cols_launch(const Tin *in, int64_t ldi, Tout *out, int64_t ldo, int64_t nrows, int ncols,
                      hipStream_t s) {
  int64_t total = nrows * ncols;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) return;
  hipLaunchKernelGGL((copy_cols_kernel<Tin, Tout>), dim3((unsigned)blocks), dim3(256), 0, s, in, ldi, out, ldo,
                     nrows, ncols);
}
template void copy_cols_launch<double, double>(const double *, int64_t, double *, int64_t, int64_t, int,
                                               hipStream_t);
template void copy_cols_launch<double, float>(const double *, int64_t, float *, int64_t, int64_t, int,
                                              hipStream_t);
template void copy_cols_launch<float, double>(const float *, int64_t, double *, int64_t, int64_t, int,
                                              hipStream_t);
template void copy_cols_launch<float, float>(const float *, int64_t, float *, int64_t, int64_t, int, hipStream_t);

// Sets *flag = 1 if any of the nrows x ncols values is NaN or Inf.
template <typename T>
__global__ __launch_bounds__(256) void nonfinite_kernel(const T *__restrict__ X, int64_t ld, int64_t nrows,
                                                        int ncols, int *flag) {
  const int64_t total = nrows * (int64_t)ncols;
  bool bad = false;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = t / ncols;
    int j = (int)(t - i * ncols);
    T v = X[i * ld + j];
    if (!(v - v == T(0))) bad = true;
  }
  if (bad) *flag = 1;
}

template <typename T>
void nonfinite_launch(const T *X, int64_t ld, int64_t nrows, int ncols, int *flag, hipStream_t s) {
  int64_t total = nrows * ncols;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) return;
  hipLaunchKernelGGL((nonfinite_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, X, ld, nrows, ncols, flag);
}
template void nonfinite_launch<double>(const double *, int64_t, int64_t, int, int *, hipStream_t);
template void nonfinite_launch<float>(const float *, int64_t, int64_t, int, int *, hipStream_t);

}  // namespace chfsi
