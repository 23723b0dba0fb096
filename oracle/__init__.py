"""FP64 CPU oracle for one energy + forces (+ virial) evaluation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C-ABI library
and its Python binding) may import, call or link anything in this package;
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP path: it has its own
neighbour search, basis functions, spherical harmonics, coupling tensors,
weight-blob parser, layer equations and analytic backward.

Scope (arxiv 2509.21694):
* the message-passing potential itself is not written down in the paper;
  the layer equations below are the reading stated in the design notes
  (NequIP/MACE style, both cited in the introduction);
* depth pruning (Methods, "Message Passing Depth Pruning"): only the first
  K of the T layers in a weight set are evaluated and the readout is taken
  from layer K;
* graph partitioning (Methods, "Graph Partitioning", stage 1 spatial grid)
  with a geometric halo, and the output integration rules of Methods
  "Global Output Integration" (energies summed over root atoms, gradients
  summed over partitions, stress by the same decomposition).

Every function is plain NumPy in float64 and follows the definitions in the
order written in its docstring; there is no autograd anywhere.
"""
from .neighbors import neighbor_list, edge_vectors            # noqa: F401
from .radial import bessel_basis, envelope, radial_features   # noqa: F401
from .sh import real_sh, real_sh_grad                          # noqa: F401
from .gaunt import gaunt_tensor, coupling_tensor, layer_paths  # noqa: F401
from .weights import parse_weights                             # noqa: F401
from .model import evaluate, Result                            # noqa: F401
from .partition import slab_share, bfs_share, hop_distance, evaluate_partitioned, local_cluster  # noqa: F401
