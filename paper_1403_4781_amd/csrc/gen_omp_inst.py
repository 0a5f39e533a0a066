"""Generate the instantiation units (omp_inst_*.hip) and the tile table (omp_table.inc) of the
fused OMP kernel.  A tile is (EM entries per lane, SM max steps, G lanes per signal, TT):
work items hold 16*TT signals.  Rerun after changing the list below."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def configs():
    out = []
    for G, EMs in ((16, (4, 8, 12, 16)), (32, (4, 8, 16)), (64, (4, 8, 16))):
        for EM in EMs:
            for SM in (8, 12, 16):
                if EM * SM > 256 and not (G == 64 and EM == 16):
                    continue          # U (EM x SM floats per lane) would not fit in registers
                if G == 16 and EM == 16 and SM == 16:
                    continue
                for TT in (1, 2, 4):
                    if EM * G * 16 * TT * 4 > 140 * 1024:
                        continue      # alpha0 staging would exceed the LDS
                    out.append((EM, SM, G, TT))
    return out


def main(nunits: int = 8):
    cfg = configs()
    units = [[] for _ in range(nunits)]
    for i, c in enumerate(cfg):
        units[i % nunits].append(c)
    for u, lst in enumerate(units):
        with open(os.path.join(HERE, f"omp_inst_{u}.hip"), "w") as f:
            f.write("// Generated instantiations of the fused OMP kernel (see omp_kernel.h).\n")
            f.write('#include "omp_kernel.h"\n\nnamespace smdl_omp {\n')
            for EM, SM, G, TT in lst:
                f.write(f"template hipError_t launch_one<{EM}, {SM}, {G}, {TT}>(const OmpArgs&, int, int, hipStream_t);\n")
            f.write("}  // namespace smdl_omp\n")
    with open(os.path.join(HERE, "omp_table.inc"), "w") as f:
        f.write("// Generated: instantiated (EM, SM, G, TT) tiles of the fused OMP kernel.\n")
        for EM, SM, G, TT in cfg:
            f.write(f"SMDL_OMP_TILE({EM}, {SM}, {G}, {TT})\n")


if __name__ == "__main__":
    main()
