// The host-side planning of libfdtd, run without a GPU.  This program compiles
// the library's host source on its own (the kernel entry points stay unresolved:
// nothing here launches a kernel or touches a device) and prints what the
// library would hand to the device, for the CPU tests to check:
//
//   host_logic worklist NX NY NZ TX ROWS SLOTS
//       the work list of one launch over the board's whole tiles of TX columns and
//       ROWS owned rows, dealt to 8 XCDs of SLOTS concurrent blocks each: one line
//       "board tx ty kb ke" per entry (board -1: an idle entry)
//   host_logic coefs NX NY NZ DX DY DZ NLX NHX NLY NHY NLZ NHZ M R KMAX DT AXIS
//       the FP32 coefficient table of one axis (Eq. 5 grading): one line per
//       coefficient kind and half (node, half node), NAXIS + 1 values each
//   host_logic matsplit NX NY NZ FILE
//       a material board's split between the plain two-step kernel and its
//       material variants, from FILE: one byte per node, x fastest, bit 1 where
//       the node's PML coefficients are rebuilt, bit 2 where an edge conducts;
//       "split S mat_ty T" then one line "rb|cd|plain tx ty kb ke" per piece
#include "fdtd_host.cpp"

#include <cstdlib>

int main(int argc, char** argv)
{
    using namespace fdtd;
    if (argc >= 8 && !strcmp(argv[1], "worklist")) {
        const int nx = atoi(argv[2]), ny = atoi(argv[3]), nz = atoi(argv[4]);
        const int tx = atoi(argv[5]), rows = atoi(argv[6]), slots = atoi(argv[7]);
        std::vector<TileRef> whole, out;
        board_tiles(0, nx, ny, nz, tx, rows, whole);
        build_work(whole, slots, out);
        for (const TileRef& t : out) printf("%d %d %d %d %d\n", t.board, t.tx, t.ty, t.kb, t.ke);
        return 0;
    }
    if (argc >= 19 && !strcmp(argv[1], "coefs")) {
        fdtd_grid_desc d{};
        d.nx = atoi(argv[2]);
        d.ny = atoi(argv[3]);
        d.nz = atoi(argv[4]);
        d.dx = atof(argv[5]);
        d.dy = atof(argv[6]);
        d.dz = atof(argv[7]);
        for (int q = 0; q < 6; ++q) d.npml[q] = atoi(argv[8 + q]);
        d.pml_m = atof(argv[14]);
        d.pml_R = atof(argv[15]);
        d.pml_kappa_max = atof(argv[16]);
        const double dt = atof(argv[17]);
        const int axis = atoi(argv[18]);
        const int n = axis == 0 ? d.nx : axis == 1 ? d.ny : d.nz;
        const std::vector<float> t = coef_table(d, axis, dt);
        for (int row = 0; row < kNumCoef * 2; ++row) {
            for (int i = 0; i <= n; ++i) printf("%.9g ", (double)t[(size_t)row * (n + 1) + i]);
            printf("\n");
        }
        return 0;
    }
    if (argc >= 6 && !strcmp(argv[1], "matsplit")) {
        const int nx = atoi(argv[2]), ny = atoi(argv[3]), nz = atoi(argv[4]);
        const size_t plane = (size_t)(nx + 1) * (ny + 1);
        std::vector<uint8_t> need(plane * (nz + 1));
        FILE* f = fopen(argv[5], "rb");
        if (!f || fread(need.data(), 1, need.size(), f) != need.size()) return 3;
        fclose(f);
        // as the class build does: plane by plane, each kind of need on its own
        int hcx = 0, hcy = 0;
        tile_counts(nx, ny, 64, owned_rows(kHybridTY, 2), &hcx, &hcy);
        std::vector<uint8_t> tile_need;
        std::vector<int32_t> pre;
        for (int k = 0; k <= nz; ++k) {
            uint8_t bits = 0;
            for (size_t n = 0; n < plane; ++n) bits |= need[k * plane + n];
            if (!bits) continue;
            if (tile_need.empty()) tile_need.assign((size_t)hcx * hcy * (nz + 1), 0);
            for (uint8_t bit = 1; bit <= 2; bit <<= 1)
                if (bits & bit) mark_tile_need(&need[k * plane], nx, ny, bit, pre, &tile_need[k], nz + 1);
        }
        MaterialSplit ms;
        split_material(nx, ny, nz, tile_need, ms);
        printf("split %d mat_ty %d\n", ms.split, ms.mat_ty);
        for (const TileRef& t : ms.rb) printf("rb %d %d %d %d\n", t.tx, t.ty, t.kb, t.ke);
        for (const TileRef& t : ms.cd) printf("cd %d %d %d %d\n", t.tx, t.ty, t.kb, t.ke);
        for (const TileRef& t : ms.plain) printf("plain %d %d %d %d\n", t.tx, t.ty, t.kb, t.ke);
        return 0;
    }
    fprintf(stderr, "usage: host_logic worklist ... | coefs ... | matsplit ...\n");
    return 2;
}
