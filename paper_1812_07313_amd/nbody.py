"""Leapfrog time integration on the GPU: every step builds the tree and
lists on the device (bhq_build_lists_device), evaluates the forces
(bhq_compute) and moves the particles (bhq_kick_drift), with the particle
state resident in device memory (torch tensors, input order).

Kick-drift-kick, as the paper's cold-collapse runs integrate (Sec. 5.2):
    v += dt/2 a;  x += dt v;  a = a(x);  v += dt/2 a.

In a periodic box (box > 0) the force is TreePM: the short-range split
kernel over the device-built lists (cells beyond rcut skipped) plus, with
pm_mesh > 0, the particle-mesh long-range force; positions are mapped back
to [0, box) after each drift.

With sort_every = k > 0 the particle state is permuted into the tree order
of every k-th build (bhq_sort_to_tree_order), so that later builds gather
their particles nearly in order; state() and accelerations() still answer
in the input order.
"""
from . import bhq


class NBody:
    """x, v: (n, 3), m: (n,) float64 arrays (host or GPU tensors); eps:
    Plummer softening; theta, ncrit, nleaf: tree parameters; kernel:
    bhq.QUAD, bhq.MONO or bhq.QUAD_SOFT; precision: bhq.FP32_OFS64 or
    bhq.FP64."""

    def __init__(self, x, v, m, eps, theta, ncrit=64, nleaf=8, kernel=bhq.QUAD,
                 precision=bhq.FP32_OFS64, stream=None, box=0.0, rs=0.0, rcut=0.0,
                 pm_mesh=0, sort_every=0):
        import torch
        self.torch = torch
        dev = torch.device("cuda")

        def tens(a, shape):
            t = torch.as_tensor(a, dtype=torch.float64, device=dev)
            return t.reshape(shape).contiguous().clone()

        n = len(m)
        self.n = n
        self.x = tens(x, (n, 3))
        self.v = tens(v, (n, 3))
        self.m = tens(m, (n,))
        self.a = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        self.pot = torch.zeros(n, dtype=torch.float64, device=dev)
        # ids[k]: input index of the particle in row k (rows move when sorted)
        self.ids = torch.arange(n, dtype=torch.int64, device=dev)
        self.sort_every = int(sort_every)
        self.nforces = 0
        self.eps = float(eps)
        self.theta, self.ncrit, self.nleaf = float(theta), int(ncrit), int(nleaf)
        self.stream = stream
        self.box, self.rs, self.rcut = float(box), float(rs), float(rcut)
        self.ctx = bhq.bhq_create(0, kernel, precision)
        self.pm = None
        if self.box > 0.0:
            bhq.bhq_set_split(self.ctx, self.rs, self.rcut, self.box)
            if pm_mesh:
                self.pm = bhq.bhq_pm_create(int(pm_mesh), self.box, self.rs)
        else:
            bhq.bhq_set_eps(self.ctx, self.eps)
        self.t = 0.0
        self.have_forces = False

    def close(self):
        if self.pm is not None:
            bhq.bhq_pm_destroy(self.pm)
            self.pm = None
        if self.ctx is not None:
            bhq.bhq_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def forces(self):
        """Tree, lists and forces at the current positions."""
        bhq.bhq_build_lists_device(self.ctx, self.x, self.m, self.theta, self.ncrit,
                                   self.nleaf, self.box, self.rcut, stream=self.stream)
        bhq.bhq_compute(self.ctx, self.stream)
        if self.sort_every > 0 and self.nforces % self.sort_every == 0:
            bhq.bhq_sort_to_tree_order(self.ctx, [self.x, self.v, self.m, self.ids],
                                       self.stream)
        self.nforces += 1
        bhq.bhq_get_result_device(self.ctx, self.a, self.pot, self.stream)
        if self.pm is not None:
            bhq.bhq_pm_compute(self.pm, self.x, self.m, self.a, self.pot, accumulate=True,
                               stream=self.stream)
        self.have_forces = True

    def step(self, dt, nsteps=1):
        """nsteps kick-drift-kick steps of size dt."""
        if not self.have_forces:
            self.forces()
        for _ in range(nsteps):
            bhq.bhq_kick_drift(self.ctx, self.x, self.v, self.a, 0.5 * dt, dt,
                               self.stream)
            if self.box > 0.0:
                bhq.bhq_wrap_periodic(self.ctx, self.x, self.box, self.stream)
            self.forces()
            bhq.bhq_kick_drift(self.ctx, None, self.v, self.a, 0.5 * dt, 0.0,
                               self.stream)
            self.t += dt

    def energies(self):
        """(K, W) at the current state (W from the last force evaluation,
        with each particle's softened self pair removed)."""
        if not self.have_forces:
            self.forces()
        return bhq.bhq_energies(self.ctx, self.m, self.v, self.pot, self.eps,
                                self.stream)

    def _input_order(self, *arrays):
        self.torch.cuda.synchronize()
        ids = self.ids.cpu().numpy()
        out = []
        for t in arrays:
            a = t.cpu().numpy()
            b = a.copy()
            b[ids] = a
            out.append(b)
        return out

    def state(self):
        """Host copies (x, v) in input order."""
        return tuple(self._input_order(self.x, self.v))

    def accelerations(self):
        """Host copies (a, pot) of the last force evaluation, in input
        order."""
        return tuple(self._input_order(self.a, self.pot))
