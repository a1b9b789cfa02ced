"""Generate EOM-CCSDT sigma-vector term tables from the ground-state CCSDT tables.

Principle.  Add non-interacting continuum spin-orbitals to the orbital
space: one virtual x for IP, one occupied x for EA, two virtual x<y for DIP,
two occupied for DEA.  Every amplitude that carries all of the continuum
labels exactly once is an EOM amplitude (IP: r_i = t_i^x, r_ij^a = t_ij^ax,
r_ijk^ab = t_ijk^abx; EA: r^a = t_x^a, ...).  Because the continuum orbitals
have no integrals, the CC residual restricted to the blocks that carry every
continuum label once is linear in those amplitudes, and equals
<mu|[H-bar, R]|0>: the EOM sigma vector (eqs 1-4 with eq 5).  Differentiating
the ground-state residual terms in that direction gives the sigma terms.

Mechanics.  For every tensor of the ground-state tables, its "R-blocks" are
the blocks in which the continuum labels sit in antisymmetric groups of the
right index space; within a group they are moved to the end (x before y),
which defines the layout of the block tensor (the group loses those slots).
A bilinear term Out += a A B contributes to an R-block of Out through the
R-block of A or of B: the continuum labels land on output letters of that
factor.  Within a sub-block (a factor group intersected with an output
group) only the trailing letters can carry them (the others are fixed by
antisymmetry), and the sign is that of moving those letters to the end of
their group, in the output and in the factor.  Summation letters never carry
a continuum label (both factors would have to be first order).

The T1 dressing contributes when R has a singles part (IP, EA): X and Y gain
a continuum row/column, which makes the dressed integrals and Fock matrix
carry first-order blocks:
  IP: dGd[p,x,r,s] = -sum_m r_m Gd[p,m,r,s],  dFd[x,q] = -sum_m r_m Fd[m,q];
  EA: dGd[p,q,r,x] = +sum_a r^a Gd[p,q,r,a],  dFd[p,x] = +sum_a r^a Fd[p,a].

The DIP and DEA R operators reach rank four (4h2p, 4p2h); their quadruples
projection comes from the linearized table in csrc/eom_quad_terms.inc, whose
direction blocks receive the continuum labels the same way.

Root blocks.  Every block tensor has a leading batch slot (space b, letter
Z) over the vectors of one Davidson block: each sigma term then processes the
whole block in one GEMM (the batch letter is an output letter of the
R-carrying factor), instead of one launch per vector.

Left-hand sigma.  The sigma program is linear in R: every term has exactly
one R-derived factor (a block tensor), the other being a ground-state
constant.  The left sigma L^T (H-bar - E_CC) is its transpose in the packed
basis, obtained in reverse mode: the terms run in reverse order, and
Out += c A B with A R-derived becomes  Abar += c' B Outbar  (Abar, Outbar the
adjoint block tensors).  The engine applies to a term's output the
antisymmetrizer P over the output's groups modulo the antisymmetry the
product already has (H); written out on the packed inner product, the
transpose of Out = c P(A B) needs c' = c |H'| / |H| with H' the antisymmetry
of the adjoint product, i.e.
  c' = c * prod_{gA, gB} |gA & gB|! / prod_{gO, gB} |gO & gB|!
over the antisymmetric letter groups of A, B and Out (the groups shared by A
and Out cancel).  Coefficients are written as exact fractions.

Usage: python -m paper_2509_14157_amd.codegen.eom_jvp  (writes csrc/eom_*_terms.inc)
"""
from __future__ import annotations

import itertools
import math
import os
import re
import sys
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "csrc")

TERM = re.compile(r"^\s*(\w+)\[(\w*)\]\s*([+-])=\s*(?:([0-9./-]+)\s*\*\s*)?(\w+)\[(\w*)\]"
                  r"(?:\s*\*\s*(\w+)\[(\w*)\])?\s*$")

VARIANTS = {
    # name: (continuum labels, their index space, R blocks as (ground-state amplitude, (nh, np)))
    "IP": (("x",), "v", (("T1", (1, 0)), ("T2", (2, 1)), ("T3", (3, 2)))),
    "EA": (("x",), "o", (("T1", (0, 1)), ("T2", (1, 2)), ("T3", (2, 3)))),
    "DIP": (("x", "y"), "v", (("T2", (2, 0)), ("T3", (3, 1)), ("T4", (4, 2)))),
    "DEA": (("x", "y"), "o", (("T2", (0, 2)), ("T3", (1, 3)), ("T4", (2, 4)))),
}

# Every R-derived tensor carries a leading batch slot (index space b) over the
# vectors of a Davidson block; its letter never occurs in the ground-state tables.
BATCH = "Z"

# The quadruples projection enters only through its linearization (a
# hand-written table): direction and image names map onto the amplitude and
# residual tensors whose continuum blocks they are.
QUAD_ALIAS = {"D2": "T2", "D3": "T3", "D4": "T4", "S2": "R2", "S3": "R3", "S4": "R4"}


def read_tables(path):
    src = open(path).read()
    tabs = {}
    for m in re.finditer(r"static const char\* const (\w+)\[\] = \{(.*?)\};", src, re.S):
        body = re.sub(r"//[^\n]*", "", m.group(2))
        tabs[m.group(1)] = re.findall(r'"([^"]*)"', body)
    return tabs


class Tensor:
    """Slot spaces plus an antisymmetry partition (list of slot lists, slot order)."""

    def __init__(self, name, spaces, groups, packed=True):
        self.name = name
        self.spaces = list(spaces)        # per slot: 'o' / 'v' / 'n'
        self.groups = [list(g) for g in groups]
        self.packed = packed              # storage packs the groups

    def spec(self):
        # storage spec of a packed tensor (groups are contiguous slot runs)
        return ",".join("".join(self.spaces[s] for s in g) for g in self.groups)


def parse_decl(d):
    name, spec = [x.strip() for x in d.split(":")]
    spaces, groups, s = [], [], 0
    for tok in [t for t in spec.split(",") if t]:
        groups.append(list(range(s, s + len(tok))))
        spaces += list(tok)
        s += len(tok)
    return Tensor(name, spaces, groups)


def parse_view(v):
    name, rest = [x.strip() for x in v.split("=")]
    par, sp = re.match(r"(\w+)\((.*)\)", rest).groups()
    spaces = [c.strip() for c in sp.split(",")]
    return name, par, spaces


def dense_sym_groups(spaces, pairs):
    """Antisymmetry of a view of a dense pair-antisymmetric tensor: a pair survives if both slots share a space."""
    groups = []
    for a, b in pairs:
        if spaces[a] == spaces[b]:
            groups.append([a, b])
        else:
            groups += [[a], [b]]
    return groups


def perm_parity(seq):
    inv = 0
    for i in range(len(seq)):
        for j in range(i + 1, len(seq)):
            if seq[i] > seq[j]:
                inv += 1
    return -1 if inv & 1 else 1


def move_to_end_sign(group_letters, moved):
    """Sign of reordering a group's letters so that `moved` (in that order) come last."""
    rest = [l for l in group_letters if l not in moved]
    target = rest + list(moved)
    pos = {l: i for i, l in enumerate(group_letters)}
    return perm_parity([pos[l] for l in target])


class Generator:
    def __init__(self, variant, cc_tables, quad_tables=None):
        self.variant = variant
        self.labels, self.space, self.rblocks = VARIANTS[variant]
        self.t = cc_tables
        self.q = quad_tables if any(a == "T4" for a, _ in self.rblocks) else None
        self.prim_decls = {}     # T-only intermediates of the quadruples table that the terms use
        self.prep = []           # their defining terms
        self.tensors = {}
        self.out_terms = []      # generated term strings
        self.decls = {}          # R-block tensor name -> spec
        self.views = []          # auxiliary views (strings)
        self.nonzero = set()     # R-block tensors known to be nonzero
        self.zero_list = []      # R-block tensors to clear before a sigma evaluation
        for d in cc_tables["kCCDecl"]:
            t = parse_decl(d)
            self.tensors[t.name] = t
        self.qdecl = {}
        if self.q is not None:
            for d in ("T4 : oooo,vvvv", "R4 : oooo,vvvv"):
                t = parse_decl(d)
                self.tensors[t.name] = t
            for d in self.q["kQDecl"]:
                t = parse_decl(d)
                self.qdecl[t.name] = d
                if t.name not in QUAD_ALIAS:
                    self.tensors[t.name] = t
        # dressed / bare integrals
        self.tensors["Gd"] = Tensor("Gd", "nnnn", [[0, 1], [2, 3]], packed=False)
        self.tensors["Fd"] = Tensor("Fd", "nn", [[0], [1]], packed=False)
        self.view_parent = {}
        for v in cc_tables["kCCViews"]:
            name, par, spaces = parse_view(v)
            if par in ("G", "F0"):
                continue  # undressed blocks only enter the energy
            groups = dense_sym_groups(spaces, [(0, 1), (2, 3)]) if par == "Gd" else [[0], [1]]
            self.tensors[name] = Tensor(name, spaces, groups, packed=False)
            self.view_parent[name] = (par, spaces)

    # ---------------------------------------------------------- R-blocks
    def assignments(self, t: Tensor):
        """All placements of the continuum labels into t's groups of the right space."""
        cand = [gi for gi, g in enumerate(t.groups) if t.spaces[g[0]] == self.space]
        out = []
        if len(self.labels) == 1:
            for g in cand:
                out.append((g,))
        else:
            for gx in cand:
                for gy in cand:
                    if gx == gy and len(t.groups[gx]) < 2:
                        continue
                    out.append((gx, gy))
        return out

    def block_name(self, t: Tensor, asg):
        return f"{t.name}_{self.variant}{''.join(str(g) for g in asg)}"

    def block_tensor(self, t: Tensor, asg):
        """Declaration of the R-block: each group loses the slots its labels occupy."""
        spaces, groups, s = [], [], 0
        count = {g: asg.count(g) for g in asg}
        for gi, g in enumerate(t.groups):
            keep = len(g) - count.get(gi, 0)
            if keep == 0:
                continue
            groups.append(list(range(s, s + keep)))
            spaces += [t.spaces[g[0]]] * keep
            s += keep
        name = self.block_name(t, asg)
        # blocks are stored packed by their antisymmetric groups (for blocks of
        # dense integral views this keeps the pair antisymmetry explicit),
        # behind a leading batch slot (space b) over the vectors of one block
        self.decls[name] = ",".join(["b"] + ["".join(spaces[x] for x in g) for g in groups])
        return name

    # ---------------------------------------------------------- dressing blocks
    def view_blocks(self):
        """First-order blocks of the dressed-integral views (IP / EA only).

        The label sits at the last slot k of its group; the block equals
        -sum_m r_m V[.., m at k, ..] (IP) or +sum_a r^a V[.., a at k, ..] (EA),
        i.e. the view with slot k's space replaced by the summed one.
        """
        if len(self.labels) != 1:
            return
        rin = self.input_name("T1")
        summed = "o" if self.space == "v" else "v"
        coef = -1 if self.space == "v" else 1
        for name, (par, spaces) in self.view_parent.items():
            t = self.tensors[name]
            allowed = ({"Gd": (0, 1), "Fd": (0,)} if self.space == "v" else {"Gd": (2, 3), "Fd": (1,)})[par]
            for asg in self.assignments(t):
                k = t.groups[asg[0]][-1]
                if k not in allowed:
                    continue
                bname = self.block_tensor(t, asg)
                letters = "pqrs"[:len(spaces)]
                src_spaces = list(spaces)
                src_spaces[k] = summed
                src = f"{par}S_{''.join(src_spaces)}"
                vdef = f"{src} = {par}({','.join(src_spaces)})"
                if vdef not in self.views:
                    self.views.append(vdef)
                out_letters = "".join(letters[j] for j in range(len(spaces)) if j != k)
                src_letters = letters[:k] + "z" + letters[k + 1:]
                op = "+=" if coef > 0 else "-="
                self.out_terms.append(f"{bname}[{BATCH}{out_letters}] {op} 1 * {rin}[{BATCH}z] * {src}[{src_letters}]")
                self.nonzero.add(bname)
                self.zero_list.append(bname)

    def input_name(self, amp):
        for a, (nh, np_) in self.rblocks:
            if a == amp:
                t = self.tensors[amp]
                asg = self.assignments(t)
                assert len(asg) == 1, (amp, asg)
                return self.block_name(t, asg[0])
        return None

    # ---------------------------------------------------------- term JVP
    def jvp(self, spec, linear=False):
        """Sigma terms of one table term.

        linear=False: a ground-state term, differentiated through every factor.
        linear=True: a term of the linearized quadruples table; only the
        direction (D2, D3, D4) and the first-order intermediates (d*) carry
        the continuum labels, the other factor is a T-only tensor.
        """
        m = TERM.match(spec)
        assert m, spec
        out, lo, sg, coef, A, la, B, lb = m.groups()
        c = float(eval(coef)) if coef else 1.0
        if sg == "-":
            c = -c
        out = QUAD_ALIAS.get(out, out)
        To = self.tensors[out]
        factors = [(A, la)] + ([(B, lb)] if B else [])
        carriers = None
        if linear:
            carriers = [fi for fi, (F, _) in enumerate(factors) if F in ("D2", "D3", "D4") or F.startswith("d")]
            assert len(carriers) == 1, spec
            factors = [(QUAD_ALIAS.get(F, F), lf) for F, lf in factors]

        def letter_groups(t, letters):
            return [[letters[s] for s in g] for g in t.groups]

        go = letter_groups(To, lo)
        ospace = [To.spaces[g[0]] for g in To.groups]
        for fi, (F, lf) in enumerate(factors):
            if carriers is not None and fi not in carriers:
                continue
            TF = self.tensors[F]
            gf = letter_groups(TF, lf)
            fspace = [TF.spaces[g[0]] for g in TF.groups]
            other = factors[1 - fi] if len(factors) == 2 else None
            # (factor group, output group) sub-blocks that can carry a label
            subs = [(h, g) for h in range(len(gf)) for g in range(len(go))
                    if fspace[h] == self.space and ospace[g] == self.space
                    and any(l in go[g] for l in gf[h])]
            for choice in itertools.product(subs, repeat=len(self.labels)):
                carried = []
                ok = True
                for i, (h, g) in enumerate(choice):
                    sub = [l for l in gf[h] if l in go[g]]
                    same = [j for j, cj in enumerate(choice) if cj == (h, g)]
                    if len(sub) < len(same):
                        ok = False
                        break
                    # labels sharing a sub-block take its trailing letters in label order
                    carried.append(sub[len(sub) - len(same) + same.index(i)])
                if not ok or len(set(carried)) != len(carried):
                    continue
                fasg = tuple(h for h, _ in choice)
                oasg = tuple(g for _, g in choice)
                fname = self.block_name(TF, fasg)
                if fname not in self.nonzero:
                    continue
                sgn = 1
                for g in set(oasg):
                    sgn *= move_to_end_sign(go[g], [carried[j] for j in range(len(carried)) if oasg[j] == g])
                for h in set(fasg):
                    sgn *= move_to_end_sign(gf[h], [carried[j] for j in range(len(carried)) if fasg[j] == h])
                oname = self.block_tensor(To, oasg)
                new_lo = BATCH + "".join(l for l in lo if l not in carried)
                new_lf = BATCH + "".join(l for l in lf if l not in carried)
                cn = c * sgn
                op = "+=" if cn > 0 else "-="
                mag = "%g" % abs(cn)
                if other is None:
                    term = f"{oname}[{new_lo}] {op} {mag} * {fname}[{new_lf}]"
                elif fi == 0:
                    term = f"{oname}[{new_lo}] {op} {mag} * {fname}[{new_lf}] * {other[0]}[{other[1]}]"
                else:
                    term = f"{oname}[{new_lo}] {op} {mag} * {other[0]}[{other[1]}] * {fname}[{new_lf}]"
                self.out_terms.append(term)
                if oname not in self.nonzero:
                    self.nonzero.add(oname)
                    self.zero_list.append(oname)

    def collect_prep(self):
        """T-only quadruples intermediates referenced by the generated terms, and their definitions."""
        used = set()
        for term in self.out_terms:
            used.update(re.findall(r"(\w+)\[", term))
        prim = [n for n in self.qdecl if n not in QUAD_ALIAS and not n.startswith("d")]
        need = [n for n in prim if n in used]
        for n in need:
            self.prim_decls[n] = self.qdecl[n].split(":")[1].strip()
        for spec in self.q["kQPrep"]:
            if TERM.match(spec).group(1) in need:
                self.prep.append(spec)

    # ---------------------------------------------------------- transpose
    def letter_groups_of(self, name, letters):
        """Antisymmetric groups (as letter lists) of a tensor of the generated terms."""
        if name in self.decls:
            toks = [t for t in self.decls[name].split(",") if t]
            groups, s = [], 0
            for tok in toks:
                groups.append(list(range(s, s + len(tok))))
                s += len(tok)
        elif name in self.tensors:
            groups = self.tensors[name].groups
        elif name.startswith("GdS_"):
            groups = dense_sym_groups(list(name[4:]), [(0, 1), (2, 3)])
        elif name.startswith("FdS_"):
            groups = [[0], [1]]
        else:
            raise KeyError(name)
        assert sum(len(g) for g in groups) == len(letters), (name, letters)
        return [[letters[x] for x in g] for g in groups]

    def adjoint_terms(self):
        """The left-hand sigma program: the generated terms transposed, in reverse order."""
        blocks = set(self.decls)
        out = []
        for t in reversed(self.out_terms):
            m = TERM.match(t)
            assert m, t
            o, lo, sg, coef, a, la, b, lb = m.groups()
            assert o in blocks, t
            c = Fraction(coef) if coef else Fraction(1)
            if sg == "-":
                c = -c
            if b is None:
                assert a in blocks, t
                x, lx, k, lk = a, la, None, None
            elif a in blocks and b not in blocks:
                x, lx, k, lk = a, la, b, lb
            elif b in blocks and a not in blocks:
                x, lx, k, lk = b, lb, a, la
            else:
                raise ValueError("term not linear in R: " + t)
            if k is not None:
                gx = self.letter_groups_of(x, lx)
                gk = self.letter_groups_of(k, lk)
                go = self.letter_groups_of(o, lo)
                num = math.prod(math.factorial(len(set(p) & set(q))) for p in gx for q in gk)
                den = math.prod(math.factorial(len(set(p) & set(q))) for p in go for q in gk)
                c = c * Fraction(num, den)
            op = "+=" if c > 0 else "-="
            mag = abs(c)
            ms = str(mag.numerator) if mag.denominator == 1 else f"{mag.numerator}/{mag.denominator}"
            if k is None:
                out.append(f"L_{x}[{lx}] {op} {ms} * L_{o}[{lo}]")
            else:
                out.append(f"L_{x}[{lx}] {op} {ms} * {k}[{lk}] * L_{o}[{lo}]")
        return out

    def generate(self):
        self.view_blocks()
        for amp, _ in self.rblocks:
            self.nonzero.add(self.input_name(amp))
            t = self.tensors[amp]
            self.block_tensor(t, self.assignments(t)[0])
        for blk in ("kCCInter2", "kCCR1", "kCCR2", "kCCInter3", "kCCR3"):
            for spec in self.t[blk]:
                self.jvp(spec)
        if self.q is not None:
            for spec in self.q["kQTerms"]:
                self.jvp(spec, linear=True)
            self.collect_prep()
        outputs = []
        for amp, _ in self.rblocks:
            res = "R" + amp[1:]
            t = self.tensors[res]
            name = self.block_name(t, self.assignments(t)[0])
            outputs.append(name)
        return outputs


def emit(variant, gen: Generator, outputs):
    v = variant
    lines = [f"// Generated by paper_2509_14157_amd/codegen/eom_jvp.py from ccsdt_terms.inc: do not edit.",
             f"// {v}-EOM-CCSDT sigma = derivative of the CCSDT residual along R placed in the",
             f"// continuum blocks (see the generator for the derivation).", ""]
    inputs = [gen.input_name(a) for a, _ in gen.rblocks]
    blocks = [nhp for _, nhp in gen.rblocks]
    lines.append(f"static const char* const kEom{v}Decl[] = {{")
    for name in sorted(gen.decls):
        lines.append(f'    "{name} : {gen.decls[name]}",')
    lines.append("};")
    lines.append(f"static const char* const kEom{v}Views[] = {{")
    for vw in gen.views:
        lines.append(f'    "{vw}",')
    if not gen.views:
        lines.append('    "",')
    lines.append("};")
    lines.append(f"// R-vector blocks in order (holes, particles) and their tensors")
    lines.append(f"static const int kEom{v}Blocks[][2] = {{" + ", ".join(f"{{{a}, {b}}}" for a, b in blocks) + "};")
    # EOM amplitude = sign * continuum-block amplitude: moving the continuum
    # operator to the end of the excitation string passes the particle
    # creators (virtual label) or the hole annihilators (occupied label)
    signs = []
    for nh, np_ in blocks:
        n_pass = np_ if gen.space == "v" else nh
        if len(gen.labels) == 2:
            # two labels: each passes the same operators
            n_pass *= 2
        signs.append(-1 if n_pass % 2 else 1)
    lines.append(f"static const int kEom{v}Sign[] = {{" + ", ".join(str(x) for x in signs) + "};")
    lines.append(f"static const char* const kEom{v}In[] = {{" + ", ".join(f'"{x}"' for x in inputs) + "};")
    lines.append(f"static const char* const kEom{v}Out[] = {{" + ", ".join(f'"{x}"' for x in outputs) + "};")
    lines.append(f"static const char* const kEom{v}Zero[] = {{")
    for z in gen.zero_list:
        lines.append(f'    "{z}",')
    lines.append("};")
    lines.append(f"static const char* const kEom{v}Terms[] = {{")
    for t in gen.out_terms:
        lines.append(f'    "{t}",')
    lines.append("};")
    lines.append(f"// T-only intermediates built once per set of amplitudes")
    lines.append(f"static const char* const kEom{v}PrimDecl[] = {{")
    for name in gen.prim_decls:
        lines.append(f'    "{name} : {gen.prim_decls[name]}",')
    if not gen.prim_decls:
        lines.append('    "",')
    lines.append("};")
    lines.append(f"static const char* const kEom{v}Prep[] = {{")
    for t in gen.prep:
        lines.append(f'    "{t}",')
    if not gen.prep:
        lines.append('    "",')
    lines.append("};")
    # left-hand sigma: adjoint block tensors, the transposed program in reverse
    # order; its input is the adjoint of the sigma blocks, its output the
    # adjoint of the R blocks (every other adjoint tensor accumulates)
    lin = ["L_" + x for x in outputs]
    lout = ["L_" + x for x in inputs]
    lines.append(f"// left-hand sigma L^T (H-bar - E_CC): the transposed program (see the generator)")
    lines.append(f"static const char* const kEom{v}LDecl[] = {{")
    for name in sorted(gen.decls):
        lines.append(f'    "L_{name} : {gen.decls[name]}",')
    lines.append("};")
    lines.append(f"static const char* const kEom{v}LIn[] = {{" + ", ".join(f'"{x}"' for x in lin) + "};")
    lines.append(f"static const char* const kEom{v}LOut[] = {{" + ", ".join(f'"{x}"' for x in lout) + "};")
    lines.append(f"static const char* const kEom{v}LZero[] = {{")
    for name in sorted(gen.decls):
        if "L_" + name not in lin:
            lines.append(f'    "L_{name}",')
    lines.append("};")
    lines.append(f"static const char* const kEom{v}LTerms[] = {{")
    for t in gen.adjoint_terms():
        lines.append(f'    "{t}",')
    lines.append("};")
    return "\n".join(lines) + "\n"


def main(variants=("IP", "EA", "DIP", "DEA")):
    tabs = read_tables(os.path.join(CSRC, "ccsdt_terms.inc"))
    quad = read_tables(os.path.join(CSRC, "eom_quad_terms.inc"))
    for v in variants:
        g = Generator(v, tabs, quad)
        outs = g.generate()
        path = os.path.join(CSRC, f"eom_{v.lower()}_terms.inc")
        with open(path, "w") as f:
            f.write(emit(v, g, outs))
        print(path, len(g.out_terms), "terms")


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ("IP", "EA", "DIP", "DEA"))
