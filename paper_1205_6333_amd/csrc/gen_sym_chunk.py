#!/usr/bin/env python3
"""Generates sym_chunk_asm.h: the hot loop of the pair-symmetric product
kernel (one chunk of 16 j-elements against two particles i per lane) as gfx950
assembly with its registers chosen for the VGPR read ports.

    python paper_1205_6333_amd/csrc/gen_sym_chunk.py

Why assembly.  On gfx950 a VALU instruction whose two multiplicand sources are
VGPRs of the same parity (v2k and v2m, or one register read twice) issues at
half the rate of one whose sources differ in parity, and an SGPR operand has
the same cost (measured on the part: 4.3 vs 2.6 cycles per wave instruction
and SIMD at four waves per SIMD).  The compiler's register allocator ignores
this; here every FP32 product of the pair terms reads one even and one odd
register, except the three squares of r^2 and the square of 1/r, which read
one register twice.

What one chunk computes is the loop body of k_pair_f32_sym (mobility.hip),
with Kahan blocks of 16 or 32 terms (one or two chunks), for the
Rotne-Prager (RPY) or Oseen tensor, in free space or with fixed-point periodic
records (PER):

  for k in 0..15 (element e = (q + k) mod 16 of the chunk, read at offset k
  of the lane's doubled view; the chunk is stored as six doubled float
  arrays px, py, pz, fx, fy, fz of 256 floats each, 1024 bytes apart):
    for the lane's particles l = 0, 1:
      d = x_l - x_e (PER: the wrapped 32-bit difference, converted)
      r2 = d.d; near pairs (r2 < thr2, tested for every group of two steps
      and masked to r2 = +inf, which makes the pair contribute zero) add
      their lanes to NL and the chunk's bit to NF
      (the projections d.F of the group's first step are issued between
      the compare and the branch on its result, which hides the branch's
      wait for the compare)
      rinv = rsq(r2); A = rinv + gamma rinv^3 (Oseen: rinv);
      Bt = rinv^3 (1 - 3 gamma rinv^2) (Oseen: rinv^3)
      Y_l += A F_e + Bt (d.F_e) d                       (i side)
      c   += A F_l + Bt (d.F_l) d                       (j side, both l)
    AJ = c (k = 0) or AJ += c of lane (q - k) mod 16 (DPP row rotation)
  then, after every chunk (blocks of 16) or every second chunk (32), per
  particle and component, the Kahan step with the block sum Y (which started
  from the negated compensation NC of the previous block):
    t = S + Y; NC = Y - (t - S); S = t.

Register map (gfx950 VGPR parity rule: products read one even, one odd):
  even: particle positions X (d = X - P with P odd), i-forces FI and chunk
  forces F (multiplied by the odd differences D), gamma (times odd rinv^3),
  thr2, the i-side block sums Y, and the products rinv^2, w, Bt, sBj, sBi
  (multiplied by odd rinv, rinv^3, dFj/dFi, D);
  odd: chunk positions P, differences D, r^2, rinv, rinv^3, A, dFj, dFi,
  m3g (times even rinv^2), the sums S and the j-side sums AJ.
Hazards observed in the order of the emitted code: a DPP source is written at
least two VALU instructions before the DPP instruction reads it; a v_rsq_f32
result is read no earlier than the instruction after next; VCC written by
v_cmp is read by v_cndmask after s_nop 1; LDS results are waited for with
lgkmcnt.  Its only memory writes are the LDS writes of the j-side rows.
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "sym_chunk_asm.h")

COMP = ("x", "y", "z")
OUT = os.environ.get("SD_GEN_OUT", OUT)
JROW_BYTES = 16 * 128 * 4     # one component of the j-side rows: 16 rows of 128 floats


class Regs:
    """Fixed register numbers; parity checked by the emitter."""

    def __init__(self):
        e = iter(range(32, 256, 2))
        o = iter(range(33, 256, 2))
        self.e, self.o = e, o
        ev = lambda: next(e)
        od = lambda: next(o)
        # pinned inputs / state (operands of the asm statement)
        self.X = [[ev() for _ in COMP] for _ in range(2)]      # x_l (even)
        self.FI = [[ev() for _ in COMP] for _ in range(2)]     # F_l (even)
        self.gamma = ev()
        self.thr2 = ev()      # compared with odd values
        self.thr2o = od()     # compared with even values
        self.inf = ev()
        self.Y = [[ev() for _ in COMP] for _ in range(2)]      # block sums / -compensation (even)
        self.m3g = od()
        self.addr = od()
        self.jaddr = od()
        self.S = [[od() for _ in COMP] for _ in range(2)]      # running sums (odd)
        self.AJ = [od() for _ in COMP]                         # j-side sums (odd)
        # temporaries of a group of two steps
        self.P = [[od() for _ in COMP] for _ in range(2)]      # chunk positions (odd)
        self.F = [[ev() for _ in COMP] for _ in range(2)]      # chunk forces (even)
        self.D = [[[od() for _ in COMP] for _ in range(2)] for _ in range(2)]   # [u][l]
        self.R2 = [[od(), ev()] for _ in range(2)]                            # [u][l]: odd, even
        self.m1 = od()
        self.m2 = ev()
        self.tmpi = [od(), od()]
        # per-pair temporaries, one set per particle l
        self.t = []
        for _ in range(2):
            self.t.append(dict(rinv=od(), rinv3=od(), A=od(), dFj=od(), dFi=od(),
                               rinv2=ev(), w=ev(), Bt=ev(), sBj=ev(), sBi=ev()))
        self.C = [[ev() for _ in COMP] for _ in range(2)]      # j-side term, two buffers (even)
        self.T = ev()                                          # Kahan temporaries
        self.TMP = od()

    def used(self):
        s = set()
        for name, v in vars(self).items():
            if name in ("e", "o"):
                continue
            stack = [v]
            while stack:
                x = stack.pop()
                if isinstance(x, int):
                    s.add(x)
                elif isinstance(x, dict):
                    stack.extend(x.values())
                elif isinstance(x, (list, tuple)):
                    stack.extend(x)
        return s


class Emit:
    def __init__(self):
        self.lines = []
        self.conflicts = 0

    def op(self, text, srcs=()):
        """srcs: the two multiplicand/operand VGPRs that must differ in parity."""
        if len(srcs) == 2 and (srcs[0] % 2) == (srcs[1] % 2):
            self.conflicts += 1
        self.lines.append(text)


def v(r):
    return "v%d" % r


def gen(tensor, per):
    R = Regs()
    E = Emit()
    t = R.t

    def load_p(g):
        for u in range(2):
            for c in range(3):
                E.op("ds_read_b32 %s, %s offset:%d" % (v(R.P[u][c]), v(R.addr),
                                                      c * 1024 + (2 * g + u) * 4))

    def dots(g, u):
        """d.F_j and d.F_i of step u of group g for both particles, with the
        deferred hand-over of the previous step's j-side term (its buffer was
        last written at least two VALU instructions before)."""
        k = 2 * g + u
        for l in range(2):
            d = R.D[u][l]
            tl = t[l]
            E.op("v_mul_f32 %s, %s, %s" % (v(tl["dFj"]), v(d[2]), v(R.F[u][2])), (d[2], R.F[u][2]))
            E.op("v_fmac_f32 %s, %s, %s" % (v(tl["dFj"]), v(d[1]), v(R.F[u][1])), (d[1], R.F[u][1]))
            E.op("v_fmac_f32 %s, %s, %s" % (v(tl["dFj"]), v(d[0]), v(R.F[u][0])), (d[0], R.F[u][0]))
            if l == 0 and k >= 2:
                prev = R.C[(k - 1) % 2]
                for c in range(3):
                    E.op("v_add_f32_dpp %s, %s, %s row_ror:%d row_mask:0xf bank_mask:0xf bound_ctrl:1"
                         % (v(R.AJ[c]), v(prev[c]), v(R.AJ[c]), (k - 1) & 15))
            E.op("v_mul_f32 %s, %s, %s" % (v(tl["dFi"]), v(d[2]), v(R.FI[l][2])), (d[2], R.FI[l][2]))
            E.op("v_fmac_f32 %s, %s, %s" % (v(tl["dFi"]), v(d[1]), v(R.FI[l][1])), (d[1], R.FI[l][1]))
            E.op("v_fmac_f32 %s, %s, %s" % (v(tl["dFi"]), v(d[0]), v(R.FI[l][0])), (d[0], R.FI[l][0]))

    def group(g):
        k0 = 2 * g
        # LDS: the group's positions (odd registers) and forces (even), the
        # forces waited for after phase 1 and the near test (loading the next
        # group's positions a group early was measured slower: 1.54 against
        # 1.45 ms per launch)
        load_p(g)
        for u in range(2):
            for c in range(3):
                E.op("ds_read_b32 %s, %s offset:%d" % (v(R.F[u][c]), v(R.addr),
                                                      (3 + c) * 1024 + (k0 + u) * 4))
        # phase 1: differences and r^2
        for u in range(2):
            E.op("s_waitcnt lgkmcnt(%d)" % (6 + 3 * (1 - u)))
            for l in range(2):
                for c in range(3):
                    if per:
                        E.op("v_sub_u32 %s, %s, %s" % (v(R.tmpi[l]), v(R.X[l][c]), v(R.P[u][c])),
                             (R.X[l][c], R.P[u][c]))
                        E.op("v_cvt_f32_i32 %s, %s" % (v(R.D[u][l][c]), v(R.tmpi[l])))
                    else:
                        E.op("v_sub_f32 %s, %s, %s" % (v(R.D[u][l][c]), v(R.X[l][c]), v(R.P[u][c])),
                             (R.X[l][c], R.P[u][c]))
            for l in range(2):
                d = R.D[u][l]
                r2 = R.R2[u][l]
                E.op("v_mul_f32 %s, %s, %s" % (v(r2), v(d[2]), v(d[2])))
                E.op("v_fmac_f32 %s, %s, %s" % (v(r2), v(d[1]), v(d[1])))
                E.op("v_fmac_f32 %s, %s, %s" % (v(r2), v(d[0]), v(d[0])))
            # near test, step by step: the minimum of the step's two pairs
            # (one odd, one even register)
            mu = R.m1 if u == 0 else R.m2
            E.op("v_min_f32 %s, %s, %s" % (v(mu), v(R.R2[u][0]), v(R.R2[u][1])),
                 (R.R2[u][0], R.R2[u][1]))
        # near test of the group's four pairs (each min reads one odd and one
        # even register)
        E.op("v_min_f32 %s, %s, %s" % (v(R.m1), v(R.m1), v(R.m2)), (R.m1, R.m2))
        E.op("v_cmp_lt_f32 vcc, %s, %s" % (v(R.m1), v(R.thr2)), (R.m1, R.thr2))
        # the projections of step 0 (they need neither r^2 nor the test) sit
        # between the compare and the branch that reads its result
        E.op("s_waitcnt lgkmcnt(0)")
        dots(g, 0)
        E.op("s_cbranch_vccz SD_SKIP%d_%%=" % g)
        # the lanes with a near pair in this group (VCC of the test)
        E.op("s_or_b64 %[nl], %[nl], vcc")
        for u in range(2):
            for l in range(2):
                r2 = R.R2[u][l]
                th = R.thr2 if r2 % 2 else R.thr2o
                E.op("v_cmp_lt_f32 vcc, %s, %s" % (v(r2), v(th)), (r2, th))
                E.op("s_nop 1")
                E.op("v_cndmask_b32 %s, %s, %s, vcc" % (v(r2), v(r2), v(R.inf)))
        # the chunk's bit: chunk 8 - cnt of the tile
        E.op("s_sub_u32 %[tmp], 8, %[cnt]")
        E.op("s_lshl_b32 %[tmp], 1, %[tmp]")
        E.op("s_or_b32 %[nf], %[nf], %[tmp]")
        E.op("SD_SKIP%d_%%=:" % g)
        # phase 2: the pair terms, step by step
        for u in range(2):
            k = k0 + u
            cbuf = R.AJ if k == 0 else R.C[k % 2]
            for l in range(2):
                E.op("v_rsq_f32 %s, %s" % (v(t[l]["rinv"]), v(R.R2[u][l])))
            if u == 1:
                dots(g, 1)
            for l in range(2):
                tl = t[l]
                E.op("v_mul_f32 %s, %s, %s" % (v(tl["rinv2"]), v(tl["rinv"]), v(tl["rinv"])))
            for l in range(2):
                tl = t[l]
                E.op("v_mul_f32 %s, %s, %s" % (v(tl["rinv3"]), v(tl["rinv2"]), v(tl["rinv"])),
                     (tl["rinv2"], tl["rinv"]))
            for l in range(2):
                tl = t[l]
                if tensor == "rpy":
                    E.op("v_fma_f32 %s, %s, %s, %s" % (v(tl["A"]), v(R.gamma), v(tl["rinv3"]), v(tl["rinv"])),
                         (R.gamma, tl["rinv3"]))
                    E.op("v_fma_f32 %s, %s, %s, 1.0" % (v(tl["w"]), v(R.m3g), v(tl["rinv2"])),
                         (R.m3g, tl["rinv2"]))
            for l in range(2):
                tl = t[l]
                if tensor == "rpy":
                    E.op("v_mul_f32 %s, %s, %s" % (v(tl["Bt"]), v(tl["rinv3"]), v(tl["w"])),
                         (tl["rinv3"], tl["w"]))
                    bt = tl["Bt"]
                else:
                    bt = None
                A = tl["A"] if tensor == "rpy" else tl["rinv"]
                tl["_A"] = A
                if tensor == "rpy":
                    E.op("v_mul_f32 %s, %s, %s" % (v(tl["sBj"]), v(bt), v(tl["dFj"])), (bt, tl["dFj"]))
                    E.op("v_mul_f32 %s, %s, %s" % (v(tl["sBi"]), v(bt), v(tl["dFi"])), (bt, tl["dFi"]))
                else:
                    # Oseen: Bt = rinv^3 (odd); sB = rinv^3 * dF needs an even partner:
                    # the products are formed from the even rinv2 instead
                    # (sB = rinv2 * (rinv * dF))
                    E.op("v_mul_f32 %s, %s, %s" % (v(tl["sBj"]), v(tl["rinv2"]), v(tl["dFj"])),
                         (tl["rinv2"], tl["dFj"]))
                    E.op("v_mul_f32 %s, %s, %s" % (v(tl["sBj"]), v(tl["sBj"]), v(tl["rinv"])),
                         (tl["sBj"], tl["rinv"]))
                    E.op("v_mul_f32 %s, %s, %s" % (v(tl["sBi"]), v(tl["rinv2"]), v(tl["dFi"])),
                         (tl["rinv2"], tl["dFi"]))
                    E.op("v_mul_f32 %s, %s, %s" % (v(tl["sBi"]), v(tl["sBi"]), v(tl["rinv"])),
                         (tl["sBi"], tl["rinv"]))
            for l in range(2):
                tl = t[l]
                d = R.D[u][l]
                A = tl["_A"]
                for c in range(3):
                    E.op("v_fmac_f32 %s, %s, %s" % (v(R.Y[l][c]), v(tl["sBj"]), v(d[c])), (tl["sBj"], d[c]))
                    E.op("v_fmac_f32 %s, %s, %s" % (v(R.Y[l][c]), v(A), v(R.F[u][c])), (A, R.F[u][c]))
            for l in range(2):
                tl = t[l]
                d = R.D[u][l]
                A = tl["_A"]
                for c in range(3):
                    if l == 0:
                        E.op("v_mul_f32 %s, %s, %s" % (v(cbuf[c]), v(tl["sBi"]), v(d[c])), (tl["sBi"], d[c]))
                    else:
                        E.op("v_fmac_f32 %s, %s, %s" % (v(cbuf[c]), v(tl["sBi"]), v(d[c])), (tl["sBi"], d[c]))
                    E.op("v_fmac_f32 %s, %s, %s" % (v(cbuf[c]), v(A), v(R.FI[l][c])), (A, R.FI[l][c]))

    for g in range(8):
        group(g)
    # hand-over of step 15's j-side term (two wait states after its last
    # write), the chunk's j-side sums to this row's slots of the tile's LDS
    # rows (components 8192 bytes apart), then the next chunk: 32 floats
    # further in the staged arrays, 16 floats further in the rows
    last = R.C[15 % 2]
    E.op("s_nop 1")
    for c in range(3):
        E.op("v_add_f32_dpp %s, %s, %s row_ror:15 row_mask:0xf bank_mask:0xf bound_ctrl:1"
             % (v(R.AJ[c]), v(last[c]), v(R.AJ[c])))
    for c in range(3):
        E.op("ds_write_b32 %s, %s offset:%d" % (v(R.jaddr), v(R.AJ[c]), c * JROW_BYTES))
    E.op("v_add_u32 %s, 128, %s" % (v(R.addr), v(R.addr)))
    E.op("v_add_u32 %s, 64, %s" % (v(R.jaddr), v(R.jaddr)))
    # Kahan step of the block sums after every chunk (kmask 0: blocks of 16
    # terms per particle) or every second chunk of the tile (kmask 1: 32
    # terms); cnt counts the tile's chunks down from 8
    E.op("s_sub_u32 %[tmp], %[cnt], 1")
    E.op("s_and_b32 %[tmp], %[tmp], %[kmask]")
    E.op("s_cmp_lg_u32 %[tmp], 0")
    E.op("s_cbranch_scc1 SD_NOKAHAN_%=")
    for l in range(2):
        for c in range(3):
            S, Y = R.S[l][c], R.Y[l][c]
            E.op("v_add_f32 %s, %s, %s" % (v(R.T), v(S), v(Y)), (S, Y))
            E.op("v_sub_f32 %s, %s, %s" % (v(R.TMP), v(R.T), v(S)), (R.T, S))
            E.op("v_sub_f32 %s, %s, %s" % (v(Y), v(Y), v(R.TMP)), (Y, R.TMP))
            E.op("v_mov_b32 %s, %s" % (v(S), v(R.T)))
    E.op("SD_NOKAHAN_%=:")
    return R, E


def c_string(lines):
    return "\n".join('    "%s\\n"' % ln for ln in lines)


def main():
    out = ["// sym_chunk_asm.h -- generated by gen_sym_chunk.py; do not edit.",
           "// One chunk of the pair-symmetric kernel in gfx950 assembly (see the",
           "// generator's docstring for what it computes and the register map).",
           "#pragma once", ""]
    regs_decl = None
    for tensor in ("rpy", "oseen"):
        for per in (False, True):
            R, E = gen(tensor, per)
            name = "SD_SYM_TILE_%s_%s" % (tensor.upper(), "PER" if per else "FREE")
            out.append("// one tile = 8 chunks; %d instructions per chunk, %d products with "
                       "same-parity sources"
                       % (sum(1 for ln in E.lines if not ln.endswith(":") and not ln.startswith("s_")),
                          E.conflicts))
            lines = (["s_mov_b32 %[cnt], 8", "SD_CHUNK_%=:"] + E.lines +
                     ["s_sub_u32 %[cnt], %[cnt], 1", "s_cmp_lg_u32 %[cnt], 0",
                      "s_cbranch_scc1 SD_CHUNK_%="])
            out.append("#define %s \\" % name)
            out.append(" \\\n".join('    "%s\\n"' % ln for ln in lines))
            out.append("")
            regs_decl = R
    R = regs_decl
    # register numbers for the asm operand constraints and clobbers
    def lst(name, xs):
        out.append("#define %s %s" % (name, ", ".join(str(x) for x in xs)))
    out.append("// pinned operand registers")
    for l in range(2):
        for c in range(3):
            out.append('#define SD_SYM_R_X%d%s "{v%d}"' % (l, COMP[c], R.X[l][c]))
            out.append('#define SD_SYM_R_FI%d%s "{v%d}"' % (l, COMP[c], R.FI[l][c]))
            out.append('#define SD_SYM_R_S%d%s "{v%d}"' % (l, COMP[c], R.S[l][c]))
            out.append('#define SD_SYM_R_Y%d%s "{v%d}"' % (l, COMP[c], R.Y[l][c]))
    for nm in ("gamma", "thr2", "thr2o", "inf", "m3g", "addr", "jaddr"):
        out.append('#define SD_SYM_R_%s "{v%d}"' % (nm.upper(), getattr(R, nm)))
    pinned = set()
    for l in range(2):
        for c in range(3):
            pinned |= {R.X[l][c], R.FI[l][c], R.S[l][c], R.Y[l][c]}
    pinned |= {R.gamma, R.thr2, R.thr2o, R.inf, R.m3g, R.addr, R.jaddr}
    clob = sorted(R.used() - pinned)
    out.append("// clobbered temporaries")
    out.append("#define SD_SYM_CLOBBERS " + ", ".join('"v%d"' % r for r in clob))
    out.append("// highest register used by the chunk: v%d" % max(R.used()))
    open(OUT, "w").write("\n".join(out) + "\n")
    print("wrote", OUT, "max reg v%d" % max(R.used()))


if __name__ == "__main__":
    main()
