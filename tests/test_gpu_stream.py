"""The torch boundary: a context bound to a PyTorch (HIP) stream with
oif_bind_stream runs its work there, and one bound to two PyTorch tensors with
oif_bind_device_buffers keeps its populations in them.  Checked in child
processes that import torch before loading liboif.so, so that both use one HIP
runtime (torch ships its own copy of it; the library then resolves to the copy
already loaded).  Stream:

* eager steps and steps replayed from a captured hipGraph on the torch stream
  give the same bits as a context on its own stream, and so do steps after
  unbinding;
* the work is ordered on that stream: with a spin kernel of known length
  queued on the torch stream first, a bound context's step (which ends by
  synchronising its stream) returns only after the spin, an unbound one
  does not wait for it.
Device buffers:

* the state is copied into the tensors when they are bound, and eager,
  graph-replayed and batched steps on them give the same bits as a context
  on buffers of its own; the steps write the tensors;
* calls with one buffer, too little memory, misaligned, overlapping, host
  memory or the bound buffers swapped are refused and change nothing;
  binding two new tensors moves the state into them;
* the FP64, FP16 and BF16 forms take buffers of their own size and give the
  same bits bound and unbound;
* unbinding copies the state back and the tensors are no longer written."""
import os
import subprocess
import sys

import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys, time
sys.path.insert(0, {root!r})
import numpy as np
import torch
torch.cuda.init()
ts = torch.cuda.Stream()
from paper_1312_3426_amd import oif, synth
oif.lib()
hips = sorted({{ln.split()[-1] for ln in open('/proc/self/maps') if 'libamdhip64' in ln}})
print('HIP runtimes loaded:', hips, flush=True)
if len(hips) != 1:
    sys.exit(3)

def state(c):
    X, V = c.read_mesh(-1)
    return [c.read_populations(), X, V]

def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))

box = synth.config_channel_rbc(30, n_cells=4)
ref = oif.Context.from_box(box, precision='fp32')
bnd = oif.Context.from_box(box, precision='fp32')
bnd.bind_stream(ts.cuda_stream)
for c in (ref, bnd):
    c.step(10)
    c.set_graph(4)
    c.step(10)
assert same(state(ref), state(bnd)), 'bound eager + graph steps differ'
print('bound eager + graph: bitwise equal', flush=True)

# spin kernel of a measured length on the torch stream
def spin(cycles):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(ts):
        e0.record(ts)
        torch.cuda._sleep(cycles)
        e1.record(ts)
    e1.synchronize()
    return e0.elapsed_time(e1)
cycles = 1 << 20
ms = spin(cycles)
while ms < 200.0 and cycles < (1 << 40):
    cycles *= 2
    ms = spin(cycles)
print(f'spin: {{cycles}} cycles = {{ms:.1f}} ms', flush=True)
assert 200.0 <= ms < 5000.0
for c, bound in ((ref, False), (bnd, True)):
    c.set_graph(0)
    with torch.cuda.stream(ts):
        torch.cuda._sleep(cycles)
    t0 = time.perf_counter()
    c.step(1)
    dt = (time.perf_counter() - t0) * 1e3
    ts.synchronize()
    print(f'step with the spin queued, bound={{bound}}: {{dt:.1f}} ms', flush=True)
    if bound:
        assert dt > 0.8 * ms, 'the bound step did not wait for the torch stream'
    else:
        assert dt < 0.5 * ms, 'the unbound step waited for the torch stream'
bnd.bind_stream(None)
ref.step(7)
bnd.step(7)
assert same(state(ref), state(bnd)), 'steps after unbinding differ'
print('after unbinding: bitwise equal', flush=True)
ref.close(); bnd.close()
print('STREAM-OK', flush=True)
"""


def test_bind_torch_stream_eager_graph_and_order(tmp_path):
    say("[stream] oif_bind_stream with a torch stream (child process)")
    env = dict(os.environ, PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-u", "-c", SCRIPT.format(root=ROOT)], env=env, capture_output=True,
                       text=True, timeout=300)
    say(r.stdout[-3000:])
    if r.returncode != 0:
        say(r.stderr[-3000:])
    assert r.returncode == 0 and "STREAM-OK" in r.stdout


BUFFERS_SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
import ctypes as C
import numpy as np
import torch
torch.cuda.init()
from paper_1312_3426_amd import oif, synth
oif.lib()
hips = sorted({{ln.split()[-1] for ln in open('/proc/self/maps') if 'libamdhip64' in ln}})
print('HIP runtimes loaded:', hips, flush=True)
if len(hips) != 1:
    sys.exit(3)

def state(c):
    X, V = c.read_mesh(-1)
    return [c.read_populations(), X, V]

def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))

box = synth.config_channel_rbc(30, n_cells=4)
ref = oif.Context.from_box(box, precision='fp32')
c = oif.Context.from_box(box, precision='fp32')
for x in (ref, c):
    x.step(5)
nb = c.population_bytes()
assert nb == 19 * ((64 * 32 * 32 + 63) // 64 * 64) * 4, nb
t0 = torch.zeros(nb, dtype=torch.uint8, device='cuda')
t1 = torch.zeros(nb, dtype=torch.uint8, device='cuda')
torch.cuda.synchronize()
c.bind_device_buffers(t0, t1)
assert int(t0.count_nonzero()) > 0 and int(t1.count_nonzero()) > 0, 'state not copied into the tensors'
for x in (ref, c):
    x.step(6)
    x.set_graph(4)
    x.step(8)
    x.set_graph(0)
assert same(state(ref), state(c)), 'steps on the bound tensors differ'
print('bound: eager + graph bitwise equal', flush=True)
b0, b1 = t0.clone(), t1.clone()
torch.cuda.synchronize()
c.step(1)
ref.step(1)
torch.cuda.synchronize()
assert not (torch.equal(b0, t0) and torch.equal(b1, t1)), 'a step did not write the tensors'

L = oif.lib()
p0, p1 = t0.data_ptr(), t1.data_ptr()
host = np.zeros(nb + 256, dtype=np.uint8)
hp = (host.ctypes.data + 255) // 256 * 256
for args, what in (((p0, None, nb), 'one buffer'), ((p0, p1, nb - 1), 'too small'),
                   ((p0 + 4, p1, nb), 'misaligned'), ((p0, p0 + 256, nb), 'overlapping'),
                   ((p0, p0, nb), 'the same buffer twice'), ((hp, p1, nb), 'host memory')):
    rc = L.oif_bind_device_buffers(c.h, args[0], args[1], args[2])
    assert rc == -1, (what, rc)  # OIF_E_ARG
    print('refused:', what, '-', L.oif_last_error(c.h).decode(), flush=True)
rc = L.oif_bind_device_buffers(c.h, p1, p0, nb)  # swapped while bound
assert rc == -1, ('swapped', rc)
print('refused: the bound buffers swapped -', L.oif_last_error(c.h).decode(), flush=True)
for x in (ref, c):
    x.step(3)
assert same(state(ref), state(c)), 'a refused call changed the state'
# rebinding moves the state into new buffers; the old ones are left alone
u0 = torch.zeros(nb, dtype=torch.uint8, device='cuda')
u1 = torch.zeros(nb, dtype=torch.uint8, device='cuda')
torch.cuda.synchronize()
c.bind_device_buffers(u0, u1)
o0, o1 = t0.clone(), t1.clone()
torch.cuda.synchronize()
for x in (ref, c):
    x.step(2)
torch.cuda.synchronize()
assert same(state(ref), state(c)), 'steps after rebinding differ'
assert torch.equal(o0, t0) and torch.equal(o1, t1), 'the replaced tensors were written'
print('rebound: bitwise equal, the replaced tensors untouched', flush=True)

bt = oif.Batch([c])
bt.step(4)
bt.close()
ref.step(4)
assert same(state(ref), state(c)), 'batched steps on the bound tensors differ'
print('bound: batched steps bitwise equal', flush=True)

c.bind_device_buffers(None, None)
assert same(state(ref), state(c)), 'unbinding changed the state'
b0, b1 = u0.clone(), u1.clone()
torch.cuda.synchronize()
for x in (ref, c):
    x.step(5)
torch.cuda.synchronize()
assert torch.equal(b0, u0) and torch.equal(b1, u1), 'the tensors were written after unbinding'
assert same(state(ref), state(c)), 'steps after unbinding differ'
print('after unbinding: bitwise equal, tensors untouched', flush=True)
ref.close(); c.close()

# every storage form: the buffer size and a bound run against an unbound one
small = synth.config_sphere_fp64(10)
for prec, size in (('fp64', 8), ('fp16', 2), ('bf16', 2)):
    r2 = oif.Context.from_box(small, precision=prec)
    c2 = oif.Context.from_box(small, precision=prec)
    nb2 = c2.population_bytes()
    assert nb2 == 19 * ((20 * 20 * 20 + 63) // 64 * 64) * size, (prec, nb2)
    v0 = torch.empty(nb2, dtype=torch.uint8, device='cuda')
    v1 = torch.empty(nb2, dtype=torch.uint8, device='cuda')
    torch.cuda.synchronize()
    for x in (r2, c2):
        x.step(3)
    c2.bind_device_buffers(v0, v1)
    for x in (r2, c2):
        x.step(4)
    assert same(state(r2), state(c2)), prec
    c2.bind_device_buffers(None, None)
    for x in (r2, c2):
        x.step(2)
    assert same(state(r2), state(c2)), prec
    print(prec, 'bound and unbound: bitwise equal', flush=True)
    r2.close(); c2.close()
print('BUFFERS-OK', flush=True)
"""


def test_bind_torch_device_buffers(tmp_path):
    say("[stream] oif_bind_device_buffers with torch tensors (child process)")
    env = dict(os.environ, PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-u", "-c", BUFFERS_SCRIPT.format(root=ROOT)], env=env,
                       capture_output=True, text=True, timeout=300)
    say(r.stdout[-3000:])
    if r.returncode != 0:
        say(r.stderr[-3000:])
    assert r.returncode == 0 and "BUFFERS-OK" in r.stdout
