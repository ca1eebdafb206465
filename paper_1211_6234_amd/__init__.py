"""MI355X-native hot path of the dipolar Heisenberg Monte Carlo method of
Stamps & Ambrose (arXiv:1211.6234): the lattice-summed dipole kernel, the
local dipolar field, checkerboard Metropolis sweeps and observables, in
hand-written HIP for gfx950 behind the C ABI of ``include/ddmc.h``.

``paper_1211_6234_amd.ddmc`` is the Python binding (argument marshalling
only); ``paper_1211_6234_amd.workloads`` draws the synthetic inputs.
"""
