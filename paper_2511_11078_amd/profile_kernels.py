"""One launch of each transform kernel on a workload, for counter collection.

Runs a plain device copy of known size first (to calibrate byte counters
such as FETCH_SIZE / WRITE_SIZE), then one forward and one adjoint per
requested degree and form.  Meant to run under ``rocprofv3 --pmc ...``:

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d out -o k -- \\
        python3 -m paper_2511_11078_amd.profile_kernels --degrees 3,0
"""
from __future__ import annotations

import argparse


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="cone_256")
    ap.add_argument("--degrees", default="3,0")
    ap.add_argument("--form", choices=["quad", "mlp"], default="quad")
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--views", type=int, default=0, help="first V views only (0 = all)")
    a = ap.parse_args()

    import torch

    from . import configs
    from .ops import Context

    wl = configs.get(a.workload)
    g = wl.geometry() if a.views <= 0 else wl.geometry().subset_views(0, a.views)
    c = torch.from_numpy(wl.volume()).cuda()
    src = torch.empty(a.copy_mib * 1024 * 1024 // 4, dtype=torch.float32, device="cuda").uniform_()
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copy {a.copy_mib} MiB done", flush=True)
    for n in (int(x) for x in a.degrees.split(",")):
        ctx = Context(n, a.form, 0)
        y = ctx.project(c, g)
        torch.cuda.synchronize()
        print(f"project degree {n} done", flush=True)
        ctx.backproject(y, g, wl.dims)
        torch.cuda.synchronize()
        print(f"backproject degree {n} done", flush=True)
        ctx.close()


if __name__ == "__main__":
    main()
