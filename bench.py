#!/usr/bin/env python3
"""Throughput of the fused moment-space LBM step on one MI355X.

Default workload: D3Q19, FP32 moment storage, 512^3 periodic, tau = 0.6,
random solenoidal initial field (|k| <= 8, rms |u| = 0.02, seed 9160).  One
"step" is one fused stream-and-collide update of every site (one kernel
launch).  Prints ONE JSON line: the main workload's MLUPS and HBM roofline
fraction (with the calibrated counter traffic when it matches the kernel
sources), the measured copy ceiling, energy per update, the D3Q27 / 16-bit /
FP64 / D3Q27h (complete Hermite basis; bound by its arithmetic, not by HBM)
variants, the error of every non-FP64 form against FP64 after 1000 steps at
the same size (with its bar: 1e-5 FP32, 1e-3 16-bit), the discrete adjoint
(192^3, checkpoints every 50 steps) and the two-component droplet (256^3,
equal phases and with contrast), and the CPU oracle baseline (D3Q19 and
D3Q27, all host cores and one).

  python bench.py [--steps K] [--warmup W] [--lattice 19|27|27h]
                  [--storage f32|f64|f16s|bf16s] [--n 512] [--no-variants]
                  [--no-adjoint] [--no-accuracy] [--no-cpu-baseline] [--copy-probe]
                  [--copy-ceilings]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline, D3Q19 512^3 FP32 vs 16-bit moments; adjoint MLUPS"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, AMD published peak
# algorithmic bytes per lattice update: the stored planes read once and
# written once (ten moments; the split-velocity form adds three 16-bit words)
BYTES_PER_LUP = {"f64": 160, "f32": 80, "f16s": 40, "bf16s": 40, "f16su": 52}
CSRC = os.path.join(ROOT, "paper_2609_09160_amd", "csrc")
KERNEL_SRCS = [os.path.join(CSRC, f) for f in ("march.hpp", "step_kernel.hpp", "lattice.hpp",
                                                "stencil.hpp", "internal.hpp", "step_f32.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_d3q19_f32_512.txt")


def kernel_hash():
    """Hash of the sources the FP32 step kernel is compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def read_traffic(n_sites):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when absent or taken on another version of the kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sha256_16") != kernel_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_input(shape, device):
    from paper_2609_09160_amd import inputs
    return inputs.solenoidal_field(shape, device=device)


def energy_reader():
    """Callable returning the GPU's accumulated energy in joules (amd-smi
    energy counter of the device torch uses), or None where unavailable."""
    try:
        import amdsmi
        import torch
        amdsmi.amdsmi_init()
        handles = amdsmi.amdsmi_get_processor_handles()
        bus = getattr(torch.cuda.get_device_properties(0), "pci_bus_id", None)
        pick = None
        for h in handles:
            bdf = amdsmi.amdsmi_get_gpu_device_bdf(h)
            if bus is not None and int(bdf.split(":")[1], 16) == int(bus):
                pick = h
        if pick is None and len(handles) == 1:
            pick = handles[0]
        if pick is None:
            return None

        def read():
            e = amdsmi.amdsmi_get_energy_count(pick)
            return e["energy_accumulator"] * e["counter_resolution"] * 1e-6
        read()
        return read
    except Exception:
        return None


def time_steps(solver, steps, warmup, energy=None):
    """ms per step (= per launch); with `energy`, also joules over the timed
    steps (None if unreadable)."""
    import torch
    solver.step(warmup)
    solver.sync()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    e0 = energy() if energy else None
    start.record(solver.stream)
    solver.step(steps)
    end.record(solver.stream)
    torch.cuda.synchronize()
    e1 = energy() if energy else None
    ms = start.elapsed_time(end) / steps
    if energy is None:
        return ms
    return ms, (e1 - e0 if e0 is not None and e1 is not None else None)


def energy_run(n, lattice, storage, seconds=2.0):
    """Energy per lattice update from the amd-smi energy counter, over a run of
    about `seconds` (the counter advances in coarse increments); None if the
    counter cannot be read or does not advance."""
    read = energy_reader()
    if read is None:
        return None
    probe = run_gpu(n, lattice, storage, 20, 5)
    steps = max(100, int(seconds / (probe["ms_per_step"] * 1e-3)))
    r = run_gpu(n, lattice, storage, steps, 10, energy=read)
    if not r.get("nJ_per_lup"):
        return None
    return {"nJ_per_lup": round(r["nJ_per_lup"], 3), "avg_power_W": round(r["avg_power_W"], 1),
            "steps": steps, "source": "amd-smi energy counter over the timed steps"}


def run_gpu(n, lattice, storage, steps, warmup, m0=None, launch=(0, 0), energy=None,
            rounding="auto"):
    import torch
    from paper_2609_09160_amd import Solver
    shape = (n, n, n)
    own = m0 is None
    if own:
        m0 = make_input(shape, "cuda")
    s = Solver(shape, 0.6, lattice=lattice, storage=storage, rounding=rounding)
    if launch != (0, 0):
        s.set_launch(*launch)
    s.set_moments(m0)
    if own:
        del m0
    joules = None
    if energy is not None:
        ms, joules = time_steps(s, steps, warmup, energy)
    else:
        ms = time_steps(s, steps, warmup)
    red = s.reduce()
    s.close()
    del s
    torch.cuda.empty_cache()
    sites = n ** 3
    mlups = sites / (ms * 1e-3) / 1e6
    gbs = BYTES_PER_LUP[storage] * sites / (ms * 1e-3) / 1e9
    out = {"mlups": mlups, "ms_per_step": ms, "algorithmic_GBs": gbs,
           "hbm_frac": gbs / HBM_PEAK_GBS, "finite": bool(all(abs(v) < 1e300 for v in red))}
    if joules:
        out["nJ_per_lup"] = joules * 1e9 / (sites * steps)
        out["avg_power_W"] = joules / (ms * 1e-3 * steps)
    return out


def stream_ceiling(n=512 ** 3, nplanes=10, reps=5):
    """The library's plain stream copy (same memory instruction forms as the
    step) of nplanes x n floats: GB/s counting read + write.  Also the number
    of bytes one launch moves, for counter calibration."""
    import ctypes
    import torch
    from paper_2609_09160_amd import _lib
    lib = _lib.load()
    a = torch.ones(nplanes * n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    args = (ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n, nplanes,
            ctypes.c_void_p(stream.cuda_stream))
    _lib.check(lib.lbfast_stream_probe(*args))
    torch.cuda.synchronize()
    st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    st.record(stream)
    for _ in range(reps):
        _lib.check(lib.lbfast_stream_probe(*args))
    en.record(stream)
    torch.cuda.synchronize()
    ms = st.elapsed_time(en) / reps
    assert torch.equal(a[:1024], b[:1024])
    del a, b
    torch.cuda.empty_cache()
    nbytes = 2 * 4 * nplanes * n
    return nbytes / (ms * 1e-3) / 1e9, ms, nbytes


def copy_ceiling(n=512 ** 3, nplanes=10, reps=5, planes=False):
    """Best-of-reps GB/s (read + write) of one of the library's two copy
    probes over nplanes x n floats: the one-shot 16-byte copy (the fastest
    copy form measured on MI355X) or, with planes=True, the ten-plane copy
    (the step's own load/store pattern, no halos, no arithmetic)."""
    import ctypes
    import torch
    from paper_2609_09160_amd import _lib
    lib = _lib.load()
    a = torch.rand(nplanes * n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    A, B, S = (ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
               ctypes.c_void_p(stream.cuda_stream))
    if planes:
        run = lambda: _lib.check(lib.lbfast_planes_probe(A, B, n, nplanes, S))  # noqa: E731
    else:
        run = lambda: _lib.check(lib.lbfast_copy_probe(A, B, nplanes * n // 4, S))  # noqa: E731
    run()
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st.record(stream)
        run()
        en.record(stream)
        torch.cuda.synchronize()
        ms = st.elapsed_time(en)
        best = ms if best is None else min(best, ms)
    assert torch.equal(a, b)
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * nplanes * n / (best * 1e-3) / 1e9


def copy_ceilings(n=512 ** 3, nplanes=10, reps=10):
    """Copies of the step's volume (nplanes x n floats read, as many written)
    by three independent routes, best of `reps` each, GB/s counting read +
    write: the library's copy probe (16-byte accesses, non-temporal stores),
    torch's copy_ between contiguous tensors (the HIP runtime's device-to-
    device memcpy), and a torch elementwise kernel (b = a * 1)."""
    import ctypes
    import torch
    from paper_2609_09160_amd import _lib
    lib = _lib.load()
    a = torch.rand(nplanes * n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    nbytes = 2 * 4 * nplanes * n

    def best(fn):
        fn()
        torch.cuda.synchronize()
        t = None
        for _ in range(reps):
            st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            st.record(stream)
            fn()
            en.record(stream)
            torch.cuda.synchronize()
            ms = st.elapsed_time(en)
            t = ms if t is None else min(t, ms)
        return round(nbytes / (t * 1e-3) / 1e9, 1)

    A, B, S = (ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
               ctypes.c_void_p(stream.cuda_stream))
    probe = lambda: _lib.check(lib.lbfast_copy_probe(A, B, nplanes * n // 4, S))  # noqa: E731
    planes = lambda: _lib.check(lib.lbfast_planes_probe(A, B, n, nplanes, S))  # noqa: E731
    out = {"bytes_read": nbytes // 2, "bytes_written": nbytes // 2,
           "library_copy_probe_GBs": best(probe),
           "library_planes_probe_GBs": best(planes)}
    # the step's marching order over a state of the same sites in each layout
    # (GB/s counting read + write of the state: 40 B per site in FP32, 20 B at
    # 16 bits); 16-bit layouts first, so that the FP32 one leaves b == a
    side = round(n ** (1 / 3))
    if side ** 3 == n and side % 128 == 0 and nplanes == 10:
        zm = {}
        for name, layout, nb in (("16bit_planes", 1, 20), ("16bit_pairs", 2, 20),
                                 ("16bit_groups_of_four", 3, 20), ("f32_planes", 0, 40)):
            run = lambda: _lib.check(lib.lbfast_zmarch_probe(  # noqa: E731
                A, B, side, side, side, layout, min(256, side), S))
            zm[name] = round(best(run) * nb / 40, 1)
        out["zmarch_copy_GBs"] = zm
    out["torch_copy_GBs"] = best(lambda: b.copy_(a))
    out["torch_elementwise_GBs"] = best(lambda: torch.mul(a, 1.0, out=b))
    assert torch.equal(a[-4096:], b[-4096:])
    del a, b
    torch.cuda.empty_cache()
    return out


ADJ_BYTES_PER_LUP = 140   # adjoint step: read lambda' 40, F 12, u(t+1) 12, u(t) 12, gF 12;
                          # write lambda 40, gF 12 (FP32)
FWD_F_BYTES_PER_LUP = 92  # forward step with a per-site force field: 40 + 12 read, 40 written


def _adjoint_times(s, n, steps, every, reps):
    """Best forward (checkpointed) and backward times over reps, in ms."""
    import torch
    m0 = torch.zeros((10, n, n, n), dtype=torch.float32, device="cuda")
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    best_f = best_b = None
    finite = True
    for _ in range(reps):
        s.set_moments(m0)
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record(s.stream)
        ckpt = s.forward_checkpointed(steps, every)
        e1.record(s.stream)
        mT = s.moments(dtype=torch.float32)
        lam = torch.zeros_like(mT)
        lam[1:4] = mT[1:4]
        torch.cuda.synchronize()
        b0, b1 = ev(), ev()
        b0.record(s.stream)
        gF, _ = s.adjoint(steps, every, ckpt, lam, want_m0=False)
        b1.record(s.stream)
        torch.cuda.synchronize()
        tf, tb = e0.elapsed_time(e1), b0.elapsed_time(b1)
        best_f = tf if best_f is None else min(best_f, tf)
        best_b = tb if best_b is None else min(best_b, tb)
        finite = finite and bool(torch.isfinite(gF).all())
        del ckpt, gF, lam, mT
    del m0
    torch.cuda.empty_cache()
    return best_f, best_b, finite


def run_adjoint(n=192, steps=500, reps=2):
    """Adjoint workload: D3Q19 FP32 n^3 periodic, tau = 0.8, from rest, per-site
    force std 1e-6 (seed 160), J = 1/2 sum |u(T)|^2.  Adjoint MLUPS = sites *
    steps / backward time.  Headline: checkpoints every 50 steps, each segment
    recomputed before it is swept; also reported with every state kept
    (checkpoint interval 1, steps x 283 MB of HBM at 192^3), where the backward
    pass runs one adjoint step per time step."""
    import torch
    from paper_2609_09160_amd import Solver, inputs
    shape = (n, n, n)
    s = Solver(shape, 0.8, storage="f32")
    F = torch.as_tensor(inputs.random_force(shape, seed=160, std=1e-6), device="cuda",
                        dtype=torch.float32)
    s.set_force_field(F)
    sites = n ** 3
    f50, b50, fin50 = _adjoint_times(s, n, steps, 50, reps)
    f1, b1, fin1 = _adjoint_times(s, n, steps, 1, reps)
    ckpt_gb = steps * s.buffer_bytes() / 1e9
    s.close()
    torch.cuda.empty_cache()
    # the backward pass recomputes every step of a segment but its last, whose
    # result is the next checkpoint (the last segment recomputes it too)
    nseg = -(-steps // 50)
    recomputed = steps - (nseg - 1)
    # the adjoint step alone: with every state kept the backward pass runs one
    # adjoint step per time step and recomputes a single forward step
    adj_step_ms = (b1 - f1 / steps) / steps
    adj_gbs = ADJ_BYTES_PER_LUP * sites / (adj_step_ms * 1e-3) / 1e9
    return {"mlups": round(sites * steps / (b50 * 1e-3) / 1e6, 1),
            "workload": f"D3Q19 FP32 {n}^3 periodic, tau=0.8, from rest, per-site force "
                        f"std 1e-6 (seed 160), J=1/2 sum|u({steps})|^2, checkpoint every 50 "
                        "steps (backward pass recomputes each segment, then sweeps it)",
            "ms_backward": round(b50, 3), "ms_forward_checkpointed": round(f50, 3),
            "backward_bytes_per_lup": round(ADJ_BYTES_PER_LUP +
                                            FWD_F_BYTES_PER_LUP * recomputed / steps, 1),
            "recomputed_steps": recomputed,
            "every_state_kept": {
                "mlups": round(sites * steps / (b1 * 1e-3) / 1e6, 1),
                "ms_backward": round(b1, 3), "ms_forward_checkpointed": round(f1, 3),
                "backward_bytes_per_lup": ADJ_BYTES_PER_LUP,
                "checkpoint_GB": round(ckpt_gb, 1)},
            "adjoint_step_ms": round(adj_step_ms, 5),
            "adjoint_step_bytes_per_lup": ADJ_BYTES_PER_LUP,
            "adjoint_step_GBs": round(adj_gbs, 1),
            "adjoint_step_hbm_frac": round(adj_gbs / HBM_PEAK_GBS, 4),
            "finite": fin1 and fin50}


TP_BYTES_PER_LUP = 128  # two-component step, FP32: the fused step 108 (moments 40, F(t) 12
                        # and phi(t+1) 4 in; moments 40 and F(t+1) 12 out); the phase
                        # update 20 (phi, u in; phi out)
TP_CONTRAST_EXTRA = 4   # with density contrast: phi(t), read by the fused step


def run_two_phase(n=256, steps=100, warmup=10, storage="f32", contrast=False):
    """Two-component workload: D3Q19 n^3 periodic, static droplet R = 40
    centred, W = 4, sigma = 0.03, D = 0.1, equal densities, tau = 1; with
    `contrast`, densities 0.5 / 1.5 and relaxation times 0.65 / 1.7 (the
    paper's layered-channel phases: per-site density and relaxation rate,
    pressure and viscous force terms)."""
    import torch
    from paper_2609_09160_amd import Solver
    shape = (n, n, n)
    z, y, x = (torch.arange(n, device="cuda", dtype=torch.float64).view(*v)
               for v in ((n, 1, 1), (1, n, 1), (1, 1, n)))
    r = torch.sqrt((x - n / 2) ** 2 + (y - n / 2) ** 2 + (z - n / 2) ** 2)
    phi = 0.5 * (1.0 - torch.tanh(2.0 * (r - 40.0) / 4.0))
    s = Solver(shape, 1.0, storage=storage,
               scale=None if storage in ("f32", "f64") else [2.0 ** -20] * 10)
    s.set_moments(torch.zeros((10, n, n, n), dtype=torch.float64, device="cuda"))
    if contrast:
        s.enable_two_phase(0.03, 4.0, 0.1, rho=(0.5, 1.5), tau=(0.65, 1.7))
    else:
        s.enable_two_phase(0.03, 4.0, 0.1)
    s.set_phase(phi)
    del phi, r
    ms = time_steps(s, steps, warmup)
    s.reduce()  # raises if the state went non-finite
    s.close()
    torch.cuda.empty_cache()
    sites = n ** 3
    bpl = TP_BYTES_PER_LUP + (TP_CONTRAST_EXTRA if contrast else 0)
    gbs = bpl * sites / (ms * 1e-3) / 1e9
    return {"mlups": round(sites / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
            "workload": f"D3Q19 {storage.upper()} {n}^3 periodic, static droplet R=40 W=4 "
                        "sigma=0.03 D=0.1, " + ("densities 0.5/1.5, tau 0.65/1.7" if contrast
                                                else "equal densities, tau=1"),
            "bytes_per_lup_algorithmic": bpl,
            "algorithmic_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}


ACCURACY_BARS = {"f32": 1e-5, "f16s": 1e-3, "bf16s": 1e-3, "f16su": 1e-3}  # u rel L2 after 1000 steps


def accuracy_vs_fp64(n, lattices, forms, steps=1000):
    """Relative L2 error of u after `steps` of the n^3 solenoidal workload for
    each (lattice, storage, rounding) of `forms`, against the same run in FP64
    on the GPU (the FP64 path is element-wise parity-checked against the FP64
    CPU oracle)."""
    import torch
    from paper_2609_09160_amd import Solver
    m0 = make_input((n, n, n), "cuda")
    out = {}
    for lat in lattices:
        s = Solver((n, n, n), 0.6, lattice=lat, storage="f64")
        s.set_moments(m0)
        s.step(steps)
        ref = s.moments()[1:4].clone()
        s.close()
        del s
        torch.cuda.empty_cache()
        rn = float(torch.linalg.vector_norm(ref))
        for st, rd in [(st, rd) for la, st, rd in forms if la == lat]:
            s = Solver((n, n, n), 0.6, lattice=lat, storage=st, rounding=rd)
            s.set_moments(m0)
            s.step(steps)
            buf = torch.empty((10, n, n, n), dtype=torch.float32, device="cuda")
            s.moments(out=buf)
            s.close()
            del s
            e = float(torch.linalg.vector_norm(buf[1:4].double() - ref)) / rn
            del buf
            torch.cuda.empty_cache()
            out[(lat, st, rd)] = e
        del ref
        torch.cuda.empty_cache()
    del m0
    torch.cuda.empty_cache()
    return out


def _time_oracle(lattice, nthreads, budget_s):
    """MLUPS of the FP64 CPU oracle on 128^3 of the solenoidal field with
    `nthreads` OpenMP threads (None: all the process may use), about
    budget_s of timed stepping after one untimed step."""
    import numpy as np
    import oracle
    from paper_2609_09160_amd import inputs
    n = 128
    shape = (n, n, n)
    default = oracle.threads()
    oracle.set_threads(nthreads or default)
    try:
        used = oracle.threads()
        o = oracle.PopulationOracle(lattice, shape, 0.6)
        o.set_moments(inputs.solenoidal_field(shape))
        o.step(1)  # warm-up
        t0 = time.perf_counter()
        o.step(1)
        one = time.perf_counter() - t0
        k = max(1, min(1000, int(budget_s / max(one, 1e-3))))
        t0 = time.perf_counter()
        o.step(k)
        dt = time.perf_counter() - t0
        assert np.isfinite(o.f).all()
    finally:
        oracle.set_threads(default)
    return {"value": round(n ** 3 * k / dt / 1e6, 3), "unit": "MLUPS", "cores": used,
            "kind": "oracle",
            "sample": f"D3Q{lattice} FP64 population oracle, {n}^3 of the same solenoidal field, "
                      f"tau=0.6, {k} timed steps after 2 untimed ({dt:.1f} s)"}


def cpu_baseline(lattice, budget_s=6.0):
    """The FP64 CPU oracle on the host cores (all of them, and one), bounded
    samples of the workload, for the benchmarked lattice and for the other
    second-order set.  The headline is the benchmarked lattice on all cores."""
    other = 27 if lattice == 19 else 19
    out = _time_oracle(lattice, None, budget_s)
    out["one_thread"] = _time_oracle(lattice, 1, budget_s)
    out[f"d3q{other}"] = _time_oracle(other, None, budget_s)
    out[f"d3q{other}"]["one_thread"] = _time_oracle(other, 1, budget_s)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--lattice", default="19", choices=("19", "27", "27h"))
    ap.add_argument("--storage", default="f32", choices=tuple(BYTES_PER_LUP))
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the short runs of D3Q27, FP64 and 16-bit storage")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the 1000-step error of each storage form against FP64")
    ap.add_argument("--tile-rows", type=int, default=0, help="launch override (0 = default)")
    ap.add_argument("--z-chunk", type=int, default=0, help="launch override (0 = default)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the library's stream copy (counter calibration)")
    ap.add_argument("--two-phase-only", action="store_true",
                    help="time only the two-component droplet workload (for counter passes)")
    ap.add_argument("--copy-ceilings", action="store_true",
                    help="only time copies of the step's volume by three routes")
    args = ap.parse_args()
    args.lattice = args.lattice if args.lattice == "27h" else int(args.lattice)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the step shards by z-slabs with a one-site moment halo; not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    if args.copy_ceilings:
        print(json.dumps(copy_ceilings()), flush=True)
        return

    if args.two_phase_only:
        print(json.dumps({"two_phase": run_two_phase(steps=args.steps, warmup=args.warmup),
                          "two_phase_contrast": run_two_phase(steps=args.steps, warmup=args.warmup,
                                                              contrast=True)}), flush=True)
        return

    if args.copy_probe:
        gbs, ms, nbytes = stream_ceiling()
        print(json.dumps({"stream_GBs": round(gbs, 1), "ms": round(ms, 4),
                          "bytes_read": nbytes // 2, "bytes_written": nbytes // 2}))
        return

    from paper_2609_09160_amd import _lib
    _lib.load()
    n = args.n
    sites = n ** 3
    main_run = run_gpu(n, args.lattice, args.storage, args.steps, args.warmup,
                       launch=(args.tile_rows, args.z_chunk))
    ms = main_run["ms_per_step"]
    value = main_run["mlups"]
    bpl = BYTES_PER_LUP[args.storage]
    achieved = bpl * sites / (ms * 1e-3) / 1e9
    traffic = None
    if (n, args.lattice, args.storage) == (512, 19, "f32"):
        traffic = read_traffic(sites)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(value / 2300.0, 2) if (n, args.lattice, args.storage) == (512, 19, "f32") else None,
        "baseline_note": "paper: 2.3 GLUPS, 1x NVIDIA A100, D3Q19 FP32 512^3 (other hardware; context)",
        "dtype": {"f64": "f64", "f32": "f32", "f16s": "f32 (fp16-scaled storage)",
                  "bf16s": "f32 (bf16-scaled storage)",
                  "f16su": "f32 (fp16-scaled storage, velocity split over two words)"}[args.storage],
        "data": "synthetic",
        "config": {"workload": f"D3Q{args.lattice} {args.storage.upper()} {n}^3 periodic, tau=0.6, "
                               "random solenoidal field |k|<=8 rms 0.02 (seed 9160)",
                   "lattice": f"D3Q{args.lattice}", "grid": [n, n, n], "storage": args.storage},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "bytes_per_lup_algorithmic": bpl},
    }
    energy = energy_run(n, args.lattice, args.storage)
    if energy is not None:
        out["energy"] = energy
    gbs, _, _ = stream_ceiling()
    out["roofline"]["measured_stream_GBs"] = round(gbs, 1)
    out["roofline"]["frac_of_measured_stream"] = round(achieved / gbs, 4)
    cgbs = copy_ceiling()
    out["roofline"]["measured_copy_GBs"] = round(cgbs, 1)
    out["roofline"]["frac_of_measured_copy"] = round(achieved / cgbs, 4)
    pgbs = copy_ceiling(planes=True)
    out["roofline"]["measured_ten_plane_copy_GBs"] = round(pgbs, 1)
    out["roofline"]["frac_of_ten_plane_copy"] = round(achieved / pgbs, 4)
    # (lattice, storage, rounding of p* and u; "auto": FP16 to nearest, BF16 stochastic)
    VARIANTS = ((27, "f32", "auto"), (19, "f16s", "auto"), (19, "f16s", "stochastic"),
                (19, "bf16s", "auto"), (19, "f16su", "auto"), (27, "f16s", "auto"),
                (27, "f16su", "auto"), (19, "f64", "auto"),
                ("27h", "f32", "auto"), ("27h", "f16s", "auto"), ("27h", "f16su", "auto"),
                ("27h", "f64", "auto"))

    def vkey(lat, st, rd):
        return f"d3q{lat}_{st}" + ("_stochastic" if rd == "stochastic" else "")

    main_form = (args.lattice, args.storage, "auto")
    var = {}
    if not args.no_variants:
        for lat, st, rd in VARIANTS:
            if (lat, st, rd) == main_form:
                continue
            r = run_gpu(n, lat, st, max(20, args.steps // 4), 5, rounding=rd)
            var[vkey(lat, st, rd)] = {"mlups": round(r["mlups"], 1),
                                      "ms_per_step": round(r["ms_per_step"], 5),
                                      "algorithmic_GBs": round(r["algorithmic_GBs"], 1),
                                      "hbm_frac": round(r["hbm_frac"], 4)}
        out["variants"] = var
    if not args.no_accuracy and args.storage != "f64":
        # every benchmarked form that is not FP64 itself, at the benchmark's size
        forms = [main_form]
        if not args.no_variants:
            forms += [f for f in VARIANTS if f[1] != "f64" and f != main_form]
        lats = list(dict.fromkeys(lat for lat, _, _ in forms))
        errs = accuracy_vs_fp64(n, lats, forms)
        for (lat, st, rd), e in errs.items():
            entry = {"u_rel_l2_vs_fp64": float(f"{e:.3g}"), "steps": 1000,
                     "bar": ACCURACY_BARS[st], "meets_bar": bool(e <= ACCURACY_BARS[st])}
            if (lat, st, rd) == main_form:
                entry["reference"] = ("the same run in FP64 on the GPU (element-wise "
                                      "parity-checked against the FP64 CPU oracle)")
                out["accuracy"] = entry
            else:
                var[vkey(lat, st, rd)]["accuracy"] = entry
    if not args.no_adjoint:
        out["adjoint"] = run_adjoint()
    if not args.no_variants:
        out["two_phase"] = run_two_phase()
        out["two_phase_contrast"] = run_two_phase(contrast=True)
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        out["cpu_baseline"] = cpu_baseline(args.lattice)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
