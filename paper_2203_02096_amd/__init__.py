"""MI355X (gfx950) docking hot path: the libmdock HIP library and its Python binding.

The package holds the C-ABI library sources (csrc/), the build script and a thin ctypes
binding whose functions carry the C names (md_eval, md_local_search, md_local_search_sw, md_local_search_traced,
md_dock, ...).
"""
from .mdock import (Ligand, MdockError, Receptor, Server, dock_params, lib, md_dock, md_dock_batch,  # noqa: F401
                    md_dock_noalloc,
                    md_dock_planned_generations, md_eval, md_ligand_info, md_local_search, md_local_search_sw, md_local_search_traced, md_pose,
                    md_profile_enable, md_profile_read, md_profile_reset,
                    md_set_graphs, md_graphs_enabled, md_ligand_get_plan, md_ligand_set_plan,
                    md_ligand_autotune, md_tune_table_clear, md_tune_table_size, md_schedule_preview,
                    md_batch_autotune, md_autogrid_map_parse, md_pdbqt_parse, md_atom_par_parse,
                    receptor_from_autogrid, ligand_from_pdbqt)
