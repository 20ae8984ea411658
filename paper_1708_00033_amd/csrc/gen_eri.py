"""Generate the per-class electron-repulsion-integral device functions.

For each of the 21 canonical quartet classes (l_a l_b | l_c l_d) with
l_a >= l_b, l_c >= l_d and bra pair class >= ket pair class (s, p and
Cartesian d shells), emit a straight-line HIP device function that

1. loops over the primitive pairs of the bra and the ket,
2. evaluates the Boys function F_m(T), m = 0..L,
3. runs the Obara-Saika vertical recurrence to [e0|f0]^(0) for
   l_a <= |e| <= l_a+l_b and l_c <= |f| <= l_c+l_d and accumulates those
   over the primitives (contraction before transfer, Head-Gordon-Pople),
4. applies the horizontal recurrence on the bra, then on the ket,
   (a, b+1_i| = (a+1_i, b| + AB_i (a, b|, to produce the contracted
   (ab|cd) block over raw Cartesian components.

The recurrences (Obara & Saika, J. Chem. Phys. 84, 3963 (1986);
Head-Gordon & Pople, J. Chem. Phys. 89, 5777 (1988)):

  [e+1_i|f]^(m) = PA_i [e|f]^(m) + WP_i [e|f]^(m+1)
                 + e_i/(2p) ([e-1_i|f]^(m) - rho/p [e-1_i|f]^(m+1))
                 + f_i/(2(p+q)) [e|f-1_i]^(m+1)
  [e|f+1_i]^(m) = QC_i [e|f]^(m) + WQ_i [e|f]^(m+1)
                 + f_i/(2q) ([e|f-1_i]^(m) - rho/q [e|f-1_i]^(m+1))
                 + e_i/(2(p+q)) [e-1_i|f]^(m+1)
  [0|0]^(m)     = K_ab K_cd 2 pi^{5/2} / (p q sqrt(p+q)) F_m(rho |PQ|^2)

The functions are templated on the real type (double or float) so the same
text yields the FP64 and FP32 evaluators.  The bra is built first (f = 0),
then the ket; the recursion direction is the axis with the smallest
non-zero exponent (fewest terms).

Usage: python gen_eri.py OUT_DIR
"""
from __future__ import annotations

import sys

PAIR_CLASSES = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
PAIR_NAMES = ["ss", "ps", "pp", "ds", "dp", "dd"]
CLASSES = [(B, K) for B in range(6) for K in range(B + 1)]
# Workgroup size per class.  LDS (the class's Boys rows plus the bra rows of
# the task) allows one workgroup per CU for most classes at ~1,200 basis
# functions, so the workgroup size sets the waves per CU: 1024 lanes where the
# kernel fits in 128 VGPRs without spilling ((ps|ss), (ds|ss): 4 waves per
# SIMD), 512 where it fits in 256, 256 for the register-heavy classes.
WG1024 = {1, 6}
WG512 = {0, 2, 3, 4, 7, 9, 10}
# Classes whose bra primitive loop runs two primitives per trip.
UNROLL2 = set()


def wg_size(cid):
    return 1024 if cid in WG1024 else (512 if cid in WG512 else 256)


def wg_alt(cid):
    """Second workgroup size, used when two workgroups of it fit in LDS
    (small molecules: short ket ranges leave 1024-lane groups idle)."""
    return 512 if cid in WG1024 else wg_size(cid)


def cart(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


def ncart(l):
    return (l + 1) * (l + 2) // 2


def sub(v, i):
    t = list(v)
    t[i] -= 1
    return tuple(t)


def add(v, i):
    t = list(v)
    t[i] += 1
    return tuple(t)


def direction(v):
    best = None
    for i in range(3):
        if v[i] > 0 and (best is None or v[i] < v[best]):
            best = i
    return best


class ClassGen:
    def __init__(self, la, lb, lc, ld, unroll2=False):
        self.la, self.lb, self.lc, self.ld = la, lb, lc, ld
        self.unroll2 = unroll2
        self.L = la + lb + lc + ld
        self.vrr_nodes = {}
        self.vrr_code = []
        self.base_used = set()
        self.nv = 0
        self.flops = 0

    # ---- vertical recurrence (inside the primitive loop) ----
    def vrr(self, e, f, m):
        key = (e, f, m)
        if key in self.vrr_nodes:
            return self.vrr_nodes[key]
        if sum(e) == 0 and sum(f) == 0:
            self.base_used.add(m)
            name = f"b{m}"
            self.vrr_nodes[key] = name
            return name
        if sum(f) == 0:
            i = direction(e)
            e1 = sub(e, i)
            t = [f"PA{i} * {self.vrr(e1, f, m)}", f"WP{i} * {self.vrr(e1, f, m + 1)}"]
            fl = 3
            if e1[i] > 0:
                e2 = sub(e1, i)
                t.append(f"R({e1[i]}) * i2p * ({self.vrr(e2, f, m)} - rp * {self.vrr(e2, f, m + 1)})")
                fl += 4
        else:
            i = direction(f)
            f1 = sub(f, i)
            t = [f"QC{i} * {self.vrr(e, f1, m)}", f"WQ{i} * {self.vrr(e, f1, m + 1)}"]
            fl = 3
            if f1[i] > 0:
                f2 = sub(f1, i)
                t.append(f"R({f1[i]}) * i2q * ({self.vrr(e, f2, m)} - rq * {self.vrr(e, f2, m + 1)})")
                fl += 4
            if e[i] > 0:
                t.append(f"R({e[i]}) * i2pq * {self.vrr(sub(e, i), f1, m + 1)}")
                fl += 2
        name = f"v{self.nv}"
        self.nv += 1
        self.flops += fl
        self.vrr_code.append(f"const R {name} = {' + '.join(t)};")
        self.vrr_nodes[key] = name
        return name

    def targets(self):
        es = [e for n in range(self.la, self.la + self.lb + 1) for e in cart(n)]
        fs = [f for n in range(self.lc, self.lc + self.ld + 1) for f in cart(n)]
        return es, fs

    # ---- horizontal recurrences (after contraction) ----
    def emit(self, fname, a_sel=None):
        """Straight-line evaluator.  a_sel = k restricts the outputs to the
        k-th Cartesian component of shell a (all b, c, d): a pass of a large
        class, with only the recurrence nodes that this pass needs."""
        acc_name = {}
        hnodes = {}
        hcode = []
        nh = [0]
        hfl = [0]

        def hb(a, b, f):
            key = (a, b, f)
            if key in hnodes:
                return hnodes[key]
            if sum(b) == 0:
                if (a, f) not in acc_name:
                    acc_name[(a, f)] = f"c_{len(acc_name)}"
                hnodes[key] = acc_name[(a, f)]
                return hnodes[key]
            i = direction(b)
            b1 = sub(b, i)
            x1 = hb(add(a, i), b1, f)
            x2 = hb(a, b1, f)
            name = f"h{nh[0]}"
            nh[0] += 1
            hfl[0] += 2
            hcode.append(f"  const R {name} = {x1} + AB{i} * {x2};")
            hnodes[key] = name
            return name

        knodes = {}

        def hk(a, b, c, d):
            key = (a, b, c, d)
            if key in knodes:
                return knodes[key]
            if sum(d) == 0:
                knodes[key] = hb(a, b, c)
                return knodes[key]
            i = direction(d)
            d1 = sub(d, i)
            x1 = hk(a, b, add(c, i), d1)
            x2 = hk(a, b, c, d1)
            name = f"h{nh[0]}"
            nh[0] += 1
            hfl[0] += 2
            hcode.append(f"  const R {name} = {x1} + CD{i} * {x2};")
            knodes[key] = name
            return name

        outs = []
        idx = 0
        alist = cart(self.la) if a_sel is None else [cart(self.la)[a_sel]]
        for a in alist:
            for b in cart(self.lb):
                for c in cart(self.lc):
                    for d in cart(self.ld):
                        outs.append(f"  out[{idx}] = {hk(a, b, c, d)};")
                        idx += 1
        # vertical recurrence for exactly the accumulators the transfers use
        for (e, f) in acc_name:
            self.vrr(e, f, 0)
        lines = []
        L = self.L
        # R: evaluation precision; SP: storage of the primitive data (the FP32
        # evaluation reads FP32 copies); TT: the Boys table rows
        lines.append("template <typename R, int BS = BOYS_ROW, typename SP = double, typename TT = R>")
        lines.append(f"__device__ __forceinline__ void {fname}(")
        lines.append("    const SP* __restrict__ bp, int nbp, const SP* __restrict__ kq0, int kfs, int kps,")
        lines.append("    int nkp, const R AB0, const R AB1, const R AB2, const R CD0, const R CD1, const R CD2,")
        lines.append("    const TT* __restrict__ boys_tab, R* __restrict__ out) {")
        for a in acc_name.values():
            lines.append(f"  R {a} = R(0);")
        lines.append("  // ket primitives (per lane, structure of arrays: field stride kfs, primitive stride kps)")
        lines.append("  for (int ik = 0; ik < nkp; ++ik) {")
        lines.append("    const SP* kq = kq0 + ik * kps;")
        lines.append("    const R q = R(kq[0]), i2q = R(kq[kfs]), Kk = R(kq[8 * kfs]);")
        lines.append("    const R Q0 = R(kq[2 * kfs]), Q1 = R(kq[3 * kfs]), Q2 = R(kq[4 * kfs]);")
        lines.append("    const R QC0 = R(kq[5 * kfs]), QC1 = R(kq[6 * kfs]), QC2 = R(kq[7 * kfs]);")
        lines.append("    // bra primitives (uniform across the workgroup)")
        # a rolled bra loop measured as fast as an unrolled one for low L (the
        # waves per SIMD hide the recurrence latency) and compiles faster
        # one bra primitive: scalar loads at a uniform address in the constant
        # address space, then the Boys function and the recurrences
        blk = ["const HFX_CONST_AS SP* B = (const HFX_CONST_AS SP*)(bp + (IB) * HFX_PRIM_FIELDS);",
               "const R p = R(B[0]), i2p = R(B[1]), Kb = R(B[8]);",
               "const R PA0 = R(B[5]), PA1 = R(B[6]), PA2 = R(B[7]);",
               "const R PQ0 = R(B[2]) - Q0, PQ1 = R(B[3]) - Q1, PQ2 = R(B[4]) - Q2;",
               "const R rs = hfx_rsqrt(p + q);   // 1/sqrt(p+q)",
               "const R ipq = rs * rs;",
               "const R rho = p * q * ipq;",
               "const R T = rho * (PQ0 * PQ0 + PQ1 * PQ1 + PQ2 * PQ2);",
               "const R pref = Kb * Kk * rs;",
               f"R F[{L + 1}];",
               f"boys_eval<R, {L}, BS>(T, F, boys_tab);"]
        body = list(self.vrr_code)
        base = [f"const R b{m} = pref * F[{m}];" for m in sorted(self.base_used)]
        if L > 0:
            blk += ["const R WP0 = -q * ipq * PQ0, WP1 = -q * ipq * PQ1, WP2 = -q * ipq * PQ2;",
                    "const R WQ0 = p * ipq * PQ0, WQ1 = p * ipq * PQ1, WQ2 = p * ipq * PQ2;",
                    "const R rp = q * ipq, rq = p * ipq, i2pq = R(0.5) * ipq;",
                    "(void)WP0; (void)WP1; (void)WP2; (void)WQ0; (void)WQ1; (void)WQ2;",
                    "(void)rp; (void)rq; (void)i2pq; (void)i2p; (void)i2q;",
                    "(void)PA0; (void)PA1; (void)PA2; (void)QC0; (void)QC1; (void)QC2;"]
        else:
            blk.append("(void)i2p; (void)i2q; (void)PA0; (void)PA1; (void)PA2; (void)QC0; (void)QC1; (void)QC2;")
        blk += base + body
        blk += [f"{a} += {self.vrr_nodes[(e, f, 0)]};" for (e, f), a in acc_name.items()]

        def emit_blk(ind, ib):
            for x in blk:
                lines.append(ind + x.replace("IB", ib))

        if self.unroll2:
            # two bra primitives per trip, in separate scopes of one straight-line
            # block, so that the scheduler interleaves their independent chains
            lines.append("    int ib = 0;")
            lines.append("#pragma unroll 1")
            lines.append("    for (; ib + 1 < nbp; ib += 2) {")
            lines.append("      {")
            emit_blk("        ", "ib")
            lines.append("      }")
            lines.append("      {")
            emit_blk("        ", "(ib + 1)")
            lines.append("      }")
            lines.append("    }")
            lines.append("    if (ib < nbp) {")
            emit_blk("      ", "ib")
            lines.append("    }")
        else:
            lines.append("#pragma unroll 1")
            lines.append("    for (int ib = 0; ib < nbp; ++ib) {")
            emit_blk("      ", "ib")
            lines.append("    }")
        lines.append("  }")
        lines.append("  (void)AB0; (void)AB1; (void)AB2; (void)CD0; (void)CD1; (void)CD2;")
        lines.extend(hcode)
        lines.extend(outs)
        lines.append("}")
        self.hrr_flops = hfl[0]
        if a_sel is None:
            # Register-tiled form: the ket's KP primitives (a compile-time count)
            # are already in registers, kv[k] = {q, 1/2q, Q, Q - C, K}; the bra
            # primitive loop is outermost (one set of scalar loads per bra
            # primitive) and the KP ket primitives inside it are unrolled, so
            # their independent Boys / recurrence chains interleave.
            kr = [f"template <typename R, int BS, int KP>\n__device__ __forceinline__ void {fname}_kr(",
                  "    const PrimPair* __restrict__ bp, int nbp, const R (&kv)[KP][9], const R AB0, const R AB1,",
                  "    const R AB2, const R CD0, const R CD1, const R CD2, const R* __restrict__ boys_tab,",
                  "    R* __restrict__ out) {"]
            for a in acc_name.values():
                kr.append(f"  R {a} = R(0);")
            kr += ["#pragma unroll 1",
                   "  for (int ib = 0; ib < nbp; ++ib) {",
                   "    const HFX_CONST_AS double* B = (const HFX_CONST_AS double*)(bp + ib);",
                   "    const R p = R(B[0]), i2p = R(B[1]), Kb = R(B[8]);",
                   "    const R PA0 = R(B[5]), PA1 = R(B[6]), PA2 = R(B[7]);",
                   "    const R P0 = R(B[2]), P1 = R(B[3]), P2 = R(B[4]);",
                   "#pragma unroll",
                   "    for (int ik = 0; ik < KP; ++ik) {",
                   "      const R q = kv[ik][0], i2q = kv[ik][1], Kk = kv[ik][8];",
                   "      const R Q0 = kv[ik][2], Q1 = kv[ik][3], Q2 = kv[ik][4];",
                   "      const R QC0 = kv[ik][5], QC1 = kv[ik][6], QC2 = kv[ik][7];",
                   "      const R PQ0 = P0 - Q0, PQ1 = P1 - Q1, PQ2 = P2 - Q2;"]
            kr += ["      " + x for x in blk[4:]]
            kr += ["    }", "  }", "  (void)AB0; (void)AB1; (void)AB2; (void)CD0; (void)CD1; (void)CD2;"]
            kr.extend(hcode)
            kr.extend(outs)
            kr.append("}")
            lines.append("")
            lines.extend(kr)
        return "\n".join(lines)


# Classes whose whole integral block is too large for registers are also
# emitted as passes, one per Cartesian component of shell a.
PASS_CLASSES = {19, 20}
# Classes that also get the register-tiled kernels (ket primitives in
# registers, blocks of bras): low total angular momentum, where the per-ket
# loads and atomics weigh most against the arithmetic.
KR_CLASSES = {0, 1, 2, 3, 4, 6, 7}


def main(out_dir):
    import os
    os.makedirs(out_dir, exist_ok=True)
    table = []
    for cid, (B, K) in enumerate(CLASSES):
        la, lb = PAIR_CLASSES[B]
        lc, ld = PAIR_CLASSES[K]
        g = ClassGen(la, lb, lc, ld, cid in UNROLL2)
        fname = f"eri_{PAIR_NAMES[B]}_{PAIR_NAMES[K]}"
        body = g.emit(fname)
        extra = []
        if cid in PASS_CLASSES:
            for k in range(ncart(la)):
                extra.append(ClassGen(la, lb, lc, ld).emit(f"{fname}_p{k}", a_sel=k))
            sw = ["template <typename R, int BS = BOYS_ROW, typename SP = double, typename TT = R>",
                  f"__device__ __forceinline__ void {fname}_pass(int k, const SP* __restrict__ bp, int nbp,",
                  "    const SP* __restrict__ kq0, int kfs, int kps, int nkp, const R AB0, const R AB1,",
                  "    const R AB2, const R CD0, const R CD1, const R CD2, const TT* __restrict__ boys_tab,",
                  "    R* __restrict__ out) {", "  switch (k) {"]
            for k in range(ncart(la)):
                sw.append(f"    case {k}: {fname}_p{k}<R, BS, SP, TT>(bp, nbp, kq0, kfs, kps, nkp, AB0, AB1, AB2, CD0, "
                          "CD1, CD2, boys_tab, out); break;")
            sw += ["    default: break;", "  }", "}"]
            extra.append("\n".join(sw))
        hdr = ["// Generated by gen_eri.py: Obara-Saika / Head-Gordon-Pople evaluator.",
               f"// class {cid}: ({PAIR_NAMES[B]}|{PAIR_NAMES[K]}), L = {g.L}", "#pragma once",
               '#include "../hfx_internal.h"', "", body, ""] + extra + [""]
        with open(os.path.join(out_dir, f"eri_class_{cid:02d}.h"), "w") as fh:
            fh.write("\n".join(hdr))
        macro = "HFX_CLASS_TU_PASSES" if cid in PASS_CLASSES else "HFX_CLASS_TU"
        tu = [f"// Generated by gen_eri.py: kernels of class {cid} ({PAIR_NAMES[B]}|{PAIR_NAMES[K]}).",
              f'#include "eri_class_{cid:02d}.h"', '#include "../eri_impl.h"', "",
              f"{macro}({cid}, {fname}, {la}, {lb}, {lc}, {ld}, {wg_size(cid)}, {wg_alt(cid)})",
              f"HFX_CLASS_KR({cid})" if cid in KR_CLASSES else f"HFX_CLASS_NO_KR({cid})", ""]
        with open(os.path.join(out_dir, f"eri_class_{cid:02d}.hip"), "w") as fh:
            fh.write("\n".join(tu))
        table.append((cid, B, K, la, lb, lc, ld, g.flops, g.hrr_flops, fname))
    parts = ["// Generated by gen_eri.py: class table.", "#pragma once", "",
             "struct EriClassInfo { int B, K, la, lb, lc, ld, vrr_flops_per_prim, hrr_flops, wgs, wgs_alt; };",
             "static const EriClassInfo kEriClassInfo[21] = {"]
    for (cid, B, K, la, lb, lc, ld, fl, hfl, fname) in table:
        parts.append(f"  {{{B}, {K}, {la}, {lb}, {lc}, {ld}, {fl}, {hfl}, {wg_size(cid)}, {wg_alt(cid)}}},  // {fname}")
    parts.append("};")
    parts.append("")
    parts.append("#define HFX_FOR_EACH_CID(X) " + " ".join(f"X({cid})" for cid in range(21)))
    parts.append("")
    with open(os.path.join(out_dir, "eri_classes.h"), "w") as fh:
        fh.write("\n".join(parts))


if __name__ == "__main__":
    main(sys.argv[1])
