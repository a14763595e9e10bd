"""Feed a seeded workload (the dataclasses of paper_2512_06173_amd.workloads, read by
attribute only) to the CPU oracle.  Test infrastructure, like the rest of oracle/."""
from oracle.oracle import Oracle


def build_oracle(w, pop_every=None):
    o = Oracle(w.shape, dx=w.dx, courant=w.courant, bc=w.bc, cpml=w.cpml)
    if w.eps is not None:
        o.set_eps(w.eps)
    if w.tls is not None and len(w.tls):
        t = w.tls
        o.add_tls(t.pos, t.sigma, t.gamma, t.omega0, t.dipole, t.rho0)
    if w.multilevel is not None and len(w.multilevel):
        m = w.multilevel
        o.add_multilevel(m.nlev, m.energies, m.mop, m.dipole, m.gphi, m.rho0, m.pos, m.sigma,
                         m.gamma)
    for s in w.plane_sources:
        o.add_plane_source(s.axis, s.index, s.comp, s.amp, s.omega, s.tau, s.t0)
    for s in w.point_sources:
        o.add_point_source(s.comp, s.ijk, s.amp, s.omega, s.tau, s.t0)
    for comp, ijk in w.probes:
        o.add_probe(comp, ijk)
    if w.flux is not None:
        o.add_flux_plane(*w.flux)
    pe = w.pop_every if pop_every is None else pop_every
    if pe:
        o.record_populations(pe)
    return o
