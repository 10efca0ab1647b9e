"""Time every compiled sweep-kernel configuration on one cavity.

    python -m paper_0809_3098_amd.tile_sweep [n ...]      (default 1024 4096)

For each n, FP64 and FP32 arithmetic, every tile shape / sweeps per launch /
threads and both tile orders (plain, XCD-banded): back-to-back relaxation sweeps of a cavity's own Poisson
problem through cavity_relax, between HIP events on the cavity's stream.
One JSON line per configuration: microseconds per sweep and the algorithmic
bandwidth (24 B per interior node and sweep in FP64, 12 B in FP32).
"""
import json
import sys

F64 = [(32, 32, 1, 256), (32, 32, 2, 256), (64, 32, 2, 512), (64, 64, 1, 1024),
       (64, 64, 2, 1024), (64, 64, 3, 1024), (64, 64, 2, 512), (64, 64, 4, 512),
       (64, 64, 4, 768), (64, 64, 4, 1024), (96, 64, 2, 1024), (96, 64, 3, 1024),
       (92, 50, 4, 1024), (84, 54, 5, 1024)]
F32 = [(32, 32, 1, 256), (32, 32, 2, 256), (64, 32, 2, 512), (64, 64, 2, 512),
       (64, 64, 2, 1024), (64, 64, 4, 1024), (64, 64, 6, 1024), (96, 64, 3, 1024),
       (96, 96, 3, 1024), (88, 56, 5, 1024), (64, 64, 4, 512), (64, 64, 6, 512)]


def main(sizes):
    import torch

    from paper_0809_3098_amd.cavity import CAVITY_MIXED, Cavity, Params

    for n in sizes:
        c = Cavity(Params(n=n, re=1e4, precision=CAVITY_MIXED))
        st = c.stream
        cells = (n - 2) ** 2
        sweeps = 480 if n <= 1024 else 120

        def us_per_sweep(arith):
            c.relax(sweeps // 4 + 1, arith=arith)          # warm-up
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            done, _ = c.relax(sweeps, arith=arith)
            e1.record(st)
            e1.synchronize()
            return e0.elapsed_time(e1) * 1e3 / done

        for arith, cfgs, nbytes in ((0, F64, 24), (1, F32, 12)):
            for xcd in (0, 1):
                for tx, ty, s, nt in cfgs:
                    if arith == 0:
                        c.set_tuning(tile_x=tx, tile_y=ty, sweeps_per_launch=s, threads=nt,
                                     xcd_bands=xcd)
                    else:
                        c.set_tuning(tile_x32=tx, tile_y32=ty, sweeps_per_launch32=s,
                                     threads32=nt, xcd_bands=xcd)
                    us = us_per_sweep(arith)
                    print(json.dumps({"n": n, "arith": "f64" if arith == 0 else "f32",
                                      "cfg": [tx, ty, s, nt], "xcd": xcd,
                                      "us_per_sweep": round(us, 3),
                                      "GBps_alg": round(nbytes * cells / us / 1e3, 1)}),
                          flush=True)
        c.close()


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [1024, 4096])
