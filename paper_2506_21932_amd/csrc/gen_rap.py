"""Build-time symbolic derivation of the stencil Galerkin triple product.

For each (fine pattern, coarsening mask) this script enumerates the influence
chains I <- u <- v <- J of the coarse operator entry A^C(I, J) (Sec. 4.3:
A^C(i,j) as the sum over fine elements u, v of R(C_i,F_u) A^F(u,v) P(F_v,C_j)),
with vertex-centred trilinear P, R = P^T, coarse X <-> fine 2X+1 on coarsened
axes and identity on the others.  It then emits one fused HIP kernel per
combination: one thread per coarse element, all 27 coarse offsets in
registers, fine rows u visited in canonical order, each chain a single fma
with compile-time weights (the paper's generated-code approach, Listing in
the supplement, re-targeted to one GPU thread per coarse element).

Accumulation order per coarse offset n (fixed here, the paper's listing
fixes none): for u = fine(I)+rho in canonical rho order,
    tmp = 0; tmp = fma(A[a][u], wP, tmp) for chains a in canonical order;
    res[n] = fma(tmp, wR(rho), res[n]).

Usage: python gen_rap.py OUTPUT.inc
"""
import itertools
import sys

OFF27 = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)]


def pattern(npts):
    out = []
    for d in OFF27:
        m = sum(abs(v) for v in d)
        if npts == 27 or (npts == 19 and m <= 2) or (npts == 7 and m <= 1):
            out.append(d)
    return out


def chains(npts, cmask):
    """Returns {rho_index: [(n_index, wR, [(a_slot, wP), ...]), ...]} for all
    (rho, n) pairs with at least one chain, n and a in canonical order."""
    A = pattern(npts)
    cm = [(cmask >> a) & 1 for a in range(3)]
    out = {}
    for ri, rho in enumerate(OFF27):
        if any((not cm[a]) and rho[a] != 0 for a in range(3)):
            continue
        wR = 1.0
        for a in range(3):
            if cm[a] and rho[a] != 0:
                wR *= 0.5
        lst = []
        for ni, n in enumerate(OFF27):
            ch = []
            for si, a_ in enumerate(A):
                ok = True
                wP = 1.0
                for ax in range(3):
                    if cm[ax]:
                        d = rho[ax] + a_[ax] - 2 * n[ax]
                        if abs(d) > 1:
                            ok = False
                            break
                        if d != 0:
                            wP *= 0.5
                    else:
                        if a_[ax] != n[ax]:
                            ok = False
                            break
                if ok:
                    ch.append((si, wP))
            if ch:
                lst.append((ni, wR, ch))
        if lst:
            out[ri] = lst
    return out


def count(npts, cmask):
    return sum(len(ch) for lst in chains(npts, cmask).values() for (_, _, ch) in lst)


# pins: Table of chain counts (3d27v restriction / interpolation) and the
# per-axis closed form for the 3d7 fine pattern
assert count(19, 7) == 1685
assert count(27, 7) == 2197
assert count(7, 7) == 5 ** 3 + 6 * 4 * 5 * 5
assert count(7, 3) == 5 ** 2 + 4 * 4 * 5 + 2 * 5 ** 2


def lit(w):
    return repr(float(w))


def emit_kernel(npts, cmask):
    name = f"k_rap_{npts}_{cmask}"
    cm = [(cmask >> a) & 1 for a in range(3)]
    L = []
    L.append(f"__global__ __launch_bounds__(256) void {name}(Grid gf, const double* __restrict__ A, long sA,")
    L.append("                                                double* __restrict__ Ac, long sAc) {")
    L.append(f"  const Grid gc{{{'gf.nx / 2' if cm[0] else 'gf.nx'}, {'gf.ny / 2' if cm[1] else 'gf.ny'}, "
             f"{'gf.nz / 2' if cm[2] else 'gf.nz'}}};")
    L.append("  // contiguous coarse lines per XCD: neighbouring lines share most of")
    L.append("  // their fine neighbourhood, which then stays in one L2")
    L.append("  const unsigned k = xcd_block(blockIdx.x, gridDim.x) * 256u + threadIdx.x;")
    L.append("  if (k >= (unsigned)gc.N()) return;")
    L.append("  const unsigned nyz = (unsigned)gc.ny * (unsigned)gc.nz;")
    L.append("  const int X = (int)(k / nyz), Y = (int)((k / (unsigned)gc.nz) % (unsigned)gc.ny), "
             "Z = (int)(k % (unsigned)gc.nz);")
    fx = "2 * X + 1" if cm[0] else "X"
    fy = "2 * Y + 1" if cm[1] else "Y"
    fz = "2 * Z + 1" if cm[2] else "Z"
    L.append(f"  const int fx = {fx}, fy = {fy}, fz = {fz};")
    L.append("  const long fyz = (long)gf.ny * gf.nz;")
    for ni in range(27):
        L.append(f"  double r{ni} = 0.0;")
    ch = chains(npts, cmask)
    for ri in sorted(ch):
        rho = OFF27[ri]
        used = sorted({si for (_, _, c) in ch[ri] for (si, _) in c})
        L.append(f"  {{  // rho = {rho}")
        L.append(f"    const int ux = fx + ({rho[0]}), uy = fy + ({rho[1]}), uz = fz + ({rho[2]});")
        L.append("    if (ux >= 0 && ux < gf.nx && uy >= 0 && uy < gf.ny && uz >= 0 && uz < gf.nz) {")
        L.append("      const long iu = ux * fyz + (long)uy * gf.nz + uz;")
        for si in used:
            L.append(f"      const double a{si} = A[{si} * sA + iu];")
        for (ni, wR, c) in ch[ri]:
            terms = " ".join(f"t = fma(a{si}, {lit(wP)}, t);" for (si, wP) in c)
            L.append(f"      {{ double t = 0.0; {terms} r{ni} = fma(t, {lit(wR)}, r{ni}); }}")
        L.append("    }")
        L.append("  }")
    for ni, n in enumerate(OFF27):
        cond = (f"X + ({n[0]}) >= 0 && X + ({n[0]}) < gc.nx && Y + ({n[1]}) >= 0 && Y + ({n[1]}) < gc.ny && "
                f"Z + ({n[2]}) >= 0 && Z + ({n[2]}) < gc.nz")
        L.append(f"  Ac[{ni} * sAc + k] = ({cond}) ? r{ni} : 0.0;")
    L.append("}")
    return name, "\n".join(L)


def main(out):
    parts = ["// Generated by gen_rap.py -- fused stencil triple products (do not edit).", ""]
    table = []
    for npts in (7, 19, 27):
        for cmask in range(1, 8):
            name, src = emit_kernel(npts, cmask)
            parts.append(src)
            parts.append("")
            table.append((npts, cmask, name, count(npts, cmask)))
    parts.append("static hipError_t rap_dispatch(int pat, int cmask, const Grid& gf, const double* A, long sA,")
    parts.append("                               double* Ac, long sAc, hipStream_t st) {")
    parts.append("  const long nc = (long)((cmask & 1) ? gf.nx / 2 : gf.nx) * ((cmask & 2) ? gf.ny / 2 : gf.ny) *")
    parts.append("                  ((cmask & 4) ? gf.nz / 2 : gf.nz);")
    parts.append("  const dim3 grid((unsigned)((nc + 255) / 256)), blk(256);")
    for npts, cmask, name, _ in table:
        parts.append(f"  if (pat == {npts} && cmask == {cmask}) {{")
        parts.append(f"    hipLaunchKernelGGL({name}, grid, blk, 0, st, gf, A, sA, Ac, sAc);")
        parts.append("    return hipGetLastError();")
        parts.append("  }")
    parts.append("  return hipErrorInvalidValue;")
    parts.append("}")
    parts.append("")
    parts.append("static int rap_chain_table(int pat, int cmask) {")
    for npts, cmask, _, cnt in table:
        parts.append(f"  if (pat == {npts} && cmask == {cmask}) return {cnt};")
    parts.append("  return -1;")
    parts.append("}")
    text = "\n".join(parts) + "\n"
    tmp = out + ".tmp"
    with open(tmp, "w") as f:
        f.write(text)
    import os
    os.replace(tmp, out)


if __name__ == "__main__":
    main(sys.argv[1])
