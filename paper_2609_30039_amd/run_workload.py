"""Run a named full-size synthetic workload for a number of time steps.

A driver for profilers: it builds the workload, steps it forward (or runs
adjoint steps against one forward state) with a fixed launch shape, and can
launch the device copy kernel on a buffer of known size, so that hardware
byte counters can be calibrated against it in the same run.

    python -m paper_2609_30039_amd.run_workload --workload lorentz_flux \\
        --dtype f32 --steps 50 --shape split,0,8 [--adjoint] [--copy-bytes N]
"""
import argparse
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="lorentz_flux")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--shape", default="auto,0,0", help="KERNEL,ROWS,KZ (kernel auto|split|fused)")
    ap.add_argument("--adjoint", action="store_true", help="time adjoint steps instead of forward steps")
    ap.add_argument("--reverse", action="store_true",
                    help="reversible mode: after the forward steps, time as many backward steps")
    ap.add_argument("--copy-bytes", type=int, default=0, help="also run the device copy kernel on this many bytes")
    ap.add_argument("--monitors", action="store_true", help="record monitors while stepping")
    ap.add_argument("--poles", type=int, default=0, help="put this pole set (3 or 16) in every dispersive box")
    args = ap.parse_args(argv)

    import torch
    from . import workloads as W
    from .sim import Simulation
    from . import binding as B

    spec = W.WORKLOADS[args.workload]()
    if (args.adjoint or args.reverse) and spec.grad_box is None:
        spec.grad_box = spec.eps_box          # a forward-only workload: the gradient over its eps box
    if args.poles:
        spec = W.with_poles(spec, W.pole_set(args.poles))
    kk, rr, zz = args.shape.split(",")
    stream = torch.cuda.current_stream().cuda_stream
    cap = max(args.steps + args.warmup + 2, spec.n_steps)
    sim = Simulation(spec, dtype=args.dtype, stream=stream, max_steps=cap, kernel=kk, tile_rows=int(rr),
                     tile_kz=int(zz), reversible=args.reverse)
    print(f"[run_workload] {args.workload} {spec.shape} {args.dtype} shape={args.shape} "
          f"{'reverse' if args.reverse else ('adjoint' if args.adjoint else 'forward')} steps={args.steps}",
          flush=True)
    sim.step(args.warmup, record=args.monitors)
    torch.cuda.synchronize()
    sim.timing(1)
    t0 = time.perf_counter()
    if args.reverse:
        sim.timing(0)
        sim.step(args.steps, record=args.monitors)
        torch.cuda.synchronize()
        sim.timing(1)
        t0 = time.perf_counter()
        sim.step_reverse(args.steps)
    elif args.adjoint:
        t = sim.steps[0]
        for _ in range(args.steps):
            sim.adjoint_begin(t + 1)
            sim.step_adjoint(1)
    else:
        sim.step(args.steps, record=args.monitors)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, n = sim.timing(2)
    print(f"[run_workload] {n} stepping launches, {ms / max(n, 1) * 1e3:.2f} us each (HIP events), "
          f"{el / args.steps * 1e6:.2f} us/step wall", flush=True)
    if args.copy_bytes:
        cms = B.fdtd_copy_probe(args.copy_bytes, 3)
        print(f"[run_workload] copy kernel {args.copy_bytes} B: {cms * 1e3:.2f} us, "
              f"{2 * args.copy_bytes / (cms * 1e-3) / 1e9:.1f} GB/s", flush=True)
    sim.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
